// Batched persistent solves (rsilu_batch.h): one workgroup owns one problem and
// runs its whole preconditioned LSQR inside one launch; the autotuner picks the
// tile of that kernel, or the plain multi-kernel path, per problem signature.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <type_traits>
#include <vector>

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "rsilu_batch.h"

namespace rsilu {
namespace {

// ------------------------------------------------------------------ descriptors

// CSR product operand; rows longer than long_thresh (listed in long_rows) are
// summed by the whole workgroup.
struct BOp {
    const int32_t *ptr, *col;
    const void *val;  // FP64 (A_hat, A_hat^T), or the preconditioner's precision (Y~, Y~^T)
    const int32_t *long_rows;
    int32_t nrows, nlong, long_thresh, pad;
};

// Triangular factor in level order: position p of level l (lev[l] <= p <
// lev[l+1]) solves row rows[p] with the entries lptr[p]..lptr[p+1] of
// lcol/lval and multiplies by ldiag[p], the reciprocal diagonal (null: unit). Values in the
// preconditioner's precision.
struct BTri {
    const int32_t *lev, *rows, *lptr, *lcol;
    const void *lval, *ldiag;
    const void *lrec;  // LevelRec<T> per position
    int32_t nlev, pad;
};

struct BOut {
    double atr, nb;
    int32_t iters, status;
    int32_t pad[2];
};

// One problem of a launch: its operators and work vectors inside its handle's
// device buffer, the caller's b and x, and its outcome slot.
struct BDesc {
    BOp A, AT;
    BTri tri[4];  // applied in this order: U^T (forward), L1^T (backward), L1 (forward), U (backward)
    const int32_t *perm;
    const double *colnorm, *b;
    double *x;
    double *xh, *z, *h, *r, *q, *v, *Mv, *w;
    void *pin, *pt0, *pt1, *pt2, *pout;  // preconditioner input, temporaries, output (its precision)
    // M_b correction of Algorithm 2 through the explicit Y~ (rows in its device order):
    // corr = 0 none, 1 cheb_K Chebyshev steps on S~ (coefficients c1 then c2; K = 0: M_b = I)
    BOp Y, YT;
    const double *cheb;
    double cheb_theta, cheb_omega;
    int32_t corr, cheb_K, k, pad2;
    void *cg, *cy, *ct, *cu, *cr, *cd, *cw, *cq;  // n: g copy, y, Y~^T product; m - n: u, r, d, w, q
    double tol;
    int32_t maxit, m, n, pad;
    BOut *out;
};

// ------------------------------------------------------------------ device code

// Every pointer of a descriptor addresses device memory; viewing it in the
// global address space makes its accesses global instructions (flat ones would
// also count against the LDS counter and serialise with LDS traffic).
#define RSILU_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ RSILU_GLOBAL T *gm(T *p)
{
    return (RSILU_GLOBAL T *)p;
}

// Value of lane (lane ^ X) within each quad of lanes, X in {1, 2}, by a DPP move
// (quad_perm [1,0,3,2] or [2,3,0,1]); no LDS round trip.
template <int X>
__device__ __forceinline__ int quad_xor(int v)
{
    static_assert(X == 1 || X == 2, "quad lanes");
    return __builtin_amdgcn_mov_dpp(v, X == 1 ? 0xB1 : 0x4E, 0xF, 0xF, false);
}
template <int X>
__device__ __forceinline__ double quad_xor(double v)
{
    const int lo = quad_xor<X>(__double2loint(v)), hi = quad_xor<X>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int X>
__device__ __forceinline__ float quad_xor(float v)
{
    return __int_as_float(quad_xor<X>(__float_as_int(v)));
}

// Sum over aligned groups of G lanes by an xor butterfly: every lane of a group
// ends with the same bits (each step adds the same two operands, commuted). The
// steps inside a quad use DPP moves, wider ones cross-lane shuffles.
template <int G, class T>
__device__ __forceinline__ T lane_sum(T v)
{
#pragma unroll
    for (int off = G / 2; off > 2; off >>= 1) v += __shfl_xor(v, off);
    if constexpr (G >= 4) v += quad_xor<2>(v);
    if constexpr (G >= 2) v += quad_xor<1>(v);
    return v;
}

// Sum over the workgroup of one value per thread. Within a wavefront the xor
// butterfly leaves every lane with the same bits (each step adds the same two
// operands, commuted); the wavefront sums are then added in index order by
// every thread, so all threads return identical values and the scalar
// recurrences that follow stay uniform.
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double *red)
{
    v = lane_sum<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) s += red[i];
    return s;
}

// y = A x by one workgroup: G lanes per row, two row groups in flight per
// thread; rows longer than long_thresh are then summed by the whole workgroup.
// The caller separates it from the producers of x and the readers of y with
// workgroup barriers.
template <int NT, int G, class T = double>
__device__ __forceinline__ void wg_spmv(const BOp &a, const T *xp, T *yp, double *red)
{
    constexpr int RPP = NT / G;
    constexpr int U = 2;
    const auto ptr = gm(a.ptr);
    const auto col = gm(a.col);
    const auto val = gm(static_cast<const T *>(a.val));
    const auto x = gm(xp);
    const auto y = gm(yp);
    const int gl = threadIdx.x % G, slot = threadIdx.x / G;
    for (int base = 0; base < a.nrows; base += U * RPP) {
        int rb[U], re[U];
        bool own[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = base + u * RPP + slot;
            rb[u] = 0;
            re[u] = 0;
            own[u] = false;
            if (row < a.nrows) {
                rb[u] = ptr[row];
                re[u] = ptr[row + 1];
                if (re[u] - rb[u] > a.long_thresh)
                    re[u] = rb[u];
                else
                    own[u] = true;
            }
        }
        T s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s[u] = (T)0;
            for (int k = rb[u] + gl; k < re[u]; k += G) s[u] += val[k] * x[col[k]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s[u] = lane_sum<G>(s[u]);
            if (own[u] && gl == 0) y[base + u * RPP + slot] = s[u];
        }
    }
    const auto longr = gm(a.long_rows);
    for (int i = 0; i < a.nlong; ++i) {
        const int row = longr[i];
        const int b = ptr[row], e = ptr[row + 1];
        T s = (T)0;
        for (int k = b + (int)threadIdx.x; k < e; k += NT) s += val[k] * x[col[k]];
        const double tot = wg_sum<NT>((double)s, red);
        if (threadIdx.x == 0) y[row] = (T)tot;
    }
}

// T x = rhs by one workgroup, level by level with one barrier per level; G
// lanes per row (G <= kRecEntries). A row's first kRecEntries entries, its
// position data and diagonal come from its LevelRec, loaded (independent loads,
// one round trip) while the previous level is solved; the two levels in flight
// alternate between two register sets, so nothing waits for those loads before
// the barrier. A level then waits only for its right-hand-side and x values.
// Entries past the record are read from the level-ordered CSR. The per-lane
// summation order is that of a plain strided loop over the row. rhs and x are
// global-memory views or LDS arrays; every x store of a level precedes the
// barrier that ends it.
template <class T, int NT, int G, class RP, class XP>
__device__ __forceinline__ void wg_trsv(const BTri &t, RP rhs, XP x)
{
    static_assert(G <= kRecEntries && kRecEntries % G == 0, "a lane's record entries");
    constexpr int RPP = NT / G;
    constexpr int E = kRecEntries / G;
    const auto lev = gm(t.lev);
    const auto rows = gm(t.rows);
    const auto lptr = gm(t.lptr);
    const auto lcol = gm(t.lcol);
    const auto lval = gm(static_cast<const T *>(t.lval));
    const auto ldiag = gm(static_cast<const T *>(t.ldiag));
    const auto rec = gm(static_cast<const LevelRec<T> *>(t.lrec));
    const bool has_diag = t.ldiag != nullptr;
    const int gl = threadIdx.x % G, slot = threadIdx.x / G;
    struct Pf {
        int row, k0, k1;
        int c[E];
        T v[E];
        T d;
    };
    auto fetch = [&](int beg, int end) {
        Pf f;
        const int p = beg + slot;
        f.row = -1;
        f.k0 = 0;
        f.k1 = 0;
        f.d = T(1);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            f.c[i] = -1;
            f.v[i] = T(0);
        }
        if (p < end) {
            const auto &r = rec[p];
            f.row = r.row;
            f.k0 = r.k0;
            f.k1 = r.k1;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                f.c[i] = r.col[gl + i * G];
                f.v[i] = r.val[gl + i * G];
            }
            f.d = r.rdiag;
        }
        return f;
    };
    auto solve = [&](const Pf &cur, int beg, int end) {
        T s = T(0), rv = T(0);
        if (cur.row >= 0) {
            rv = rhs[cur.row];
#pragma unroll
            for (int i = 0; i < E; ++i)
                if (cur.c[i] >= 0) s += cur.v[i] * x[cur.c[i]];
            for (int k = cur.k0 + kRecEntries + gl; k < cur.k1; k += G) s += lval[k] * x[lcol[k]];
        }
        s = lane_sum<G>(s);
        if (cur.row >= 0 && gl == 0) {
            T r = rv - s;
            if (has_diag) r = r * cur.d;
            x[cur.row] = r;
        }
        // further rows of a level wider than one pass
        for (int base = beg + RPP; base < end; base += RPP) {
            const int p = base + slot;
            T s2 = T(0);
            int row = -1;
            if (p < end) {
                row = rows[p];
                const int k1 = lptr[p + 1];
                for (int k = lptr[p] + gl; k < k1; k += G) s2 += lval[k] * x[lcol[k]];
            }
            s2 = lane_sum<G>(s2);
            if (row >= 0 && gl == 0) {
                T r = rhs[row] - s2;
                if (has_diag) r = r * ldiag[p];
                x[row] = r;
            }
        }
    };
    __syncthreads();  // rhs complete
    const int nlev = t.nlev;
    if (nlev == 0) return;
    // Level pointers come from a window of 64 held in the lanes of every
    // wavefront (vector loads, read out with readlane): a scalar load in flight
    // would be waited for at every barrier with the LDS operations.
    const int lane = threadIdx.x & 63;
    int wbase = 0;
    int win = lev[min(lane, nlev)];
    auto lev_at = [&](int i) {
        if (i - wbase >= 64) {
            wbase = i;
            win = lev[min(wbase + lane, nlev)];
        }
        return __builtin_amdgcn_readlane(win, i - wbase);
    };
    int b0 = 0, b1 = lev_at(1);
    Pf A = fetch(b0, b1), B;
    for (int l = 0;;) {
        int b2 = l + 2 <= nlev ? lev_at(l + 2) : b1;
        B = fetch(b1, b2);
        solve(A, b0, b1);
        __syncthreads();
        if (++l == nlev) break;
        b0 = b1;
        b1 = b2;
        b2 = l + 2 <= nlev ? lev_at(l + 2) : b1;
        A = fetch(b1, b2);
        solve(B, b0, b1);
        __syncthreads();
        if (++l == nlev) break;
        b0 = b1;
        b1 = b2;
    }
}

// Steps 2-4 of Algorithm 2 with the explicit Y~ (Section 3.2), from g = L1^{-T} U^{-T} z
// (global, n values) to y = g - Y~^T v_b: w_b = Y~ g, v_b = M_b^{-1} w_b by cheb_K
// Chebyshev steps on S~ = I + Y~ Y~^T (none: v_b = w_b; per step q = Y~ (Y~^T d), w += d,
// r -= d + q, d = c1 d + c2 r, from r = omega w_b, d = r / theta, w = 0; v_b = w), then
// y = g - Y~^T v_b. The (m - n)-vectors are in the device order of Y~'s rows. The caller
// separates g's producers and y's readers from it with barriers.
template <class T, int NT, int G>
__device__ __forceinline__ void wg_correction(const BDesc &d, const T *gp, T *yp, double *red)
{
    const int n = d.n, k = d.k;
    const auto g = gm(gp);
    const auto y = gm(yp);
    T *u = static_cast<T *>(d.cu);
    T *t = static_cast<T *>(d.ct);
    wg_spmv<NT, G, T>(d.Y, gp, u, red);
    __syncthreads();
    if (d.cheb_K > 0) {
        const auto uu = gm(u);
        const auto r = gm(static_cast<T *>(d.cr)), dd = gm(static_cast<T *>(d.cd)), w = gm(static_cast<T *>(d.cw));
        const auto q = gm(static_cast<const T *>(d.cq));
        const T theta = (T)d.cheb_theta, omega = (T)d.cheb_omega;
        for (int i = threadIdx.x; i < k; i += NT) {
            const T ri = omega * uu[i];
            r[i] = ri;
            dd[i] = ri / theta;
            w[i] = (T)0;
        }
        const auto cf = gm(d.cheb);
        for (int j = 0; j < d.cheb_K; ++j) {
            __syncthreads();
            wg_spmv<NT, G, T>(d.YT, static_cast<const T *>(d.cd), t, red);
            __syncthreads();
            wg_spmv<NT, G, T>(d.Y, t, static_cast<T *>(d.cq), red);
            __syncthreads();
            const T c1 = (T)cf[j], c2 = (T)cf[d.cheb_K + j];
            const bool last = j + 1 == d.cheb_K;
            for (int i = threadIdx.x; i < k; i += NT) {
                const T di = dd[i];
                const T wi = w[i] + di;
                const T ri = r[i] - (di + q[i]);
                w[i] = wi;
                r[i] = ri;
                dd[i] = c1 * di + c2 * ri;
                if (last) uu[i] = wi;
            }
        }
        __syncthreads();
    }
    wg_spmv<NT, G, T>(d.YT, u, t, red);
    __syncthreads();
    const auto tt = gm(static_cast<const T *>(t));
    for (int i = threadIdx.x; i < n; i += NT) y[i] = g[i] - tt[i];
    __syncthreads();
}

// h = M^{-1} z with M^{-1} = (L1 U)^{-1} (L1 U)^{-T} (Algorithm 2, k = n, without the M_b
// correction): U^T t0 = z, L1^T t1 = t0, L1 t2 = t1, U h = t2; with it, t1 is replaced
// by t1 - Y~^T v_b before the L1 solve (wg_correction). In FP32 the input
// is rounded to FP32 first and h converted back. With XL the four solution
// vectors live in LDS (two arrays of n values, used alternately; xl holds 2n
// values), so a level reads its inputs from LDS instead of through the caches.
template <class T, int NT, int G, int GS, bool XL>
__device__ __forceinline__ void wg_precond_in(const BDesc &d, T *xl, double *red)
{
    const int n = d.n;
    const auto z = gm(d.z);
    const auto h = gm(d.h);
    if constexpr (std::is_same<T, float>::value) {
        const auto fi = gm(static_cast<float *>(d.pin));
        for (int i = threadIdx.x; i < n; i += NT) fi[i] = (float)z[i];
    }
    const auto in = gm(std::is_same<T, float>::value ? static_cast<const T *>(d.pin)
                                                     : reinterpret_cast<const T *>(d.z));
    if constexpr (XL) {
        T *xa = xl, *xb = xl + n;
        wg_trsv<T, NT, G>(d.tri[0], in, xa);
        wg_trsv<T, NT, G>(d.tri[1], xa, xb);
        if (d.corr) {
            __syncthreads();
            const auto gc = gm(static_cast<T *>(d.cg));
            for (int i = threadIdx.x; i < n; i += NT) gc[i] = xb[i];
            __syncthreads();
            wg_correction<T, NT, GS>(d, static_cast<const T *>(d.cg), static_cast<T *>(d.cy), red);
            wg_trsv<T, NT, G>(d.tri[2], gm(static_cast<const T *>(d.cy)), xa);
        } else {
            wg_trsv<T, NT, G>(d.tri[2], xb, xa);
        }
        wg_trsv<T, NT, G>(d.tri[3], xa, xb);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += NT) h[i] = (double)xb[i];
        __syncthreads();
    } else {
        const auto t0 = gm(static_cast<T *>(d.pt0));
        const auto t1 = gm(static_cast<T *>(d.pt1));
        const auto t2 = gm(static_cast<T *>(d.pt2));
        const auto out = gm(std::is_same<T, float>::value ? static_cast<T *>(d.pout) : reinterpret_cast<T *>(d.h));
        wg_trsv<T, NT, G>(d.tri[0], in, t0);
        wg_trsv<T, NT, G>(d.tri[1], t0, t1);
        if (d.corr) {
            __syncthreads();
            wg_correction<T, NT, GS>(d, static_cast<const T *>(d.pt1), static_cast<T *>(d.cy), red);
            wg_trsv<T, NT, G>(d.tri[2], gm(static_cast<const T *>(d.cy)), t2);
        } else {
            wg_trsv<T, NT, G>(d.tri[2], t1, t2);
        }
        wg_trsv<T, NT, G>(d.tri[3], t2, out);
        __syncthreads();
        if constexpr (std::is_same<T, float>::value)
            for (int i = threadIdx.x; i < n; i += NT) h[i] = (double)out[i];
    }
}

// The preconditioner of one problem: its solution vectors in LDS when 2 n values
// fit in the launch's dynamic LDS (xl_bytes), else in global memory.
template <class T, int NT, int G, int GS>
__device__ __forceinline__ void wg_precond(const BDesc &d, T *xl, uint32_t xl_bytes, double *red)
{
    if (2 * (uint64_t)d.n * sizeof(T) <= xl_bytes)
        wg_precond_in<T, NT, G, GS, true>(d, xl, red);
    else
        wg_precond_in<T, NT, G, GS, false>(d, xl, red);
}

// The whole LSQR solve of problem blockIdx.x (M-inner-product form): init,
// iterations until the stop test or maxit, then x = D x_hat and the true
// ||A^T (b - A x)||. Every scalar is computed identically by every thread.
template <class T, int NT, int GS, int GT>
__global__ __launch_bounds__(NT) void k_batch_lsqr(const BDesc *__restrict__ descs, uint32_t xl_bytes)
{
    __shared__ double red[NT / 64];
    extern __shared__ __attribute__((aligned(16))) unsigned char xl_lds[];  // xl_bytes: 2 n values of T
    T *xl = reinterpret_cast<T *>(xl_lds);
    const BDesc &d = descs[blockIdx.x];
    const int tid = threadIdx.x, m = d.m, n = d.n;
    const auto r = gm(d.r), q = gm(d.q), z = gm(d.z), h = gm(d.h), xh = gm(d.xh), v = gm(d.v), Mv = gm(d.Mv),
               w = gm(d.w);
    const auto bb = gm(d.b);
    const auto perm = gm(d.perm);
    const auto colnorm = gm(d.colnorm);
    const auto xo = gm(d.x);

    // u = P b / beta1 (u kept in r), x_hat = 0
    double sq = 0.0;
    for (int i = tid; i < m; i += NT) {
        const double bi = bb[perm[i]];
        r[i] = bi;
        sq += bi * bi;
    }
    for (int i = tid; i < n; i += NT) xh[i] = 0.0;
    const double b1 = sqrt(wg_sum<NT>(sq, red));
    int done = 0, status = 0, iter = 0;
    double nb = 0.0, lb = b1, la = 0.0, phibar = b1, rhobar = 0.0, snorm = 0.0;
    if (b1 == 0.0) {
        done = 1;
    } else if (!isfinite(b1)) {
        done = 1;
        status = 2;
    }
    // s = A_hat^T u, ||D^{-1} s|| gives ||A^T b|| = beta1 ||D^{-1} s||
    if (!done) {
        for (int i = tid; i < m; i += NT) r[i] = r[i] / lb;
        __syncthreads();
        wg_spmv<NT, GS>(d.AT, d.r, d.z, red);
        __syncthreads();
        sq = 0.0;
        for (int i = tid; i < n; i += NT) {
            const double c = colnorm[i] * z[i];
            sq += c * c;
        }
        snorm = sqrt(wg_sum<NT>(sq, red));
        nb = lb * snorm;
        if (nb == 0.0) {
            done = 1;
        } else if (!isfinite(nb)) {
            done = 1;
            status = 2;
        }
    }
    // h = M^{-1} s, alpha = sqrt(s . h), v = h / alpha, M v = s / alpha, w = v
    if (!done) {
        wg_precond<T, NT, GT, GS>(d, xl, xl_bytes, red);
        sq = 0.0;
        for (int i = tid; i < n; i += NT) sq += z[i] * h[i];
        const double tot = wg_sum<NT>(sq, red);
        if (!(tot > 0.0) || !isfinite(tot)) {
            done = 1;
            status = 2;
        } else {
            la = sqrt(tot);
            rhobar = la;
        }
        if (d.maxit == 0 && !done) {
            done = 1;
            status = 1;
        }
    }
    if (!done)
        for (int i = tid; i < n; i += NT) {
            const double vi = h[i] / la;
            v[i] = vi;
            Mv[i] = z[i] / la;
            w[i] = vi;
        }

    while (!done) {
        // t = A_hat v - alpha u, beta = ||t||, u = t / beta (t kept in q)
        __syncthreads();
        wg_spmv<NT, GS>(d.A, d.v, d.q, red);
        __syncthreads();
        sq = 0.0;
        for (int i = tid; i < m; i += NT) {
            const double ti = q[i] - la * r[i];
            q[i] = ti;
            sq += ti * ti;
        }
        lb = sqrt(wg_sum<NT>(sq, red));
        if (!isfinite(lb)) {
            status = 2;
            break;
        }
        for (int i = tid; i < m; i += NT) r[i] = lb > 0.0 ? q[i] / lb : q[i];
        // s = A_hat^T u - beta M v with ||D^{-1} s||
        __syncthreads();
        wg_spmv<NT, GS>(d.AT, d.r, d.z, red);
        __syncthreads();
        sq = 0.0;
        for (int i = tid; i < n; i += NT) {
            const double si = z[i] - lb * Mv[i];
            z[i] = si;
            const double c = colnorm[i] * si;
            sq += c * c;
        }
        snorm = sqrt(wg_sum<NT>(sq, red));
        // h = M^{-1} s, alpha = sqrt(s . h)
        wg_precond<T, NT, GT, GS>(d, xl, xl_bytes, red);
        sq = 0.0;
        for (int i = tid; i < n; i += NT) sq += z[i] * h[i];
        const double tot = wg_sum<NT>(sq, red);
        // plane rotation and the stop test on |phibar c| ||D^{-1} s||
        const double lan = tot > 0.0 ? sqrt(tot) : 0.0;
        const double rho = sqrt(rhobar * rhobar + lb * lb);
        const double c = rhobar / rho, sn = lb / rho;
        const double theta = sn * lan;
        rhobar = -c * lan;
        const double phi = c * phibar;
        phibar = sn * phibar;
        const double phi_rho = phi / rho, theta_rho = theta / rho;
        la = lan;
        iter += 1;
        const double est = fabs(phibar * c) * snorm;
        int lstop = 0, lstatus = 0;
        if (!isfinite(est) || !isfinite(tot) || !isfinite(rho)) {
            lstop = 1;
            lstatus = 2;
        } else if (est <= d.tol * nb) {
            lstop = 1;
        } else if (la == 0.0) {
            lstop = 1;
            lstatus = tot < 0.0 ? 2 : 0;
        } else if (iter >= d.maxit) {
            lstop = 1;
            lstatus = 1;
        }
        // x_hat += (phi / rho) w; v = h / alpha, M v = s / alpha, w = v - (theta / rho) w
        for (int i = tid; i < n; i += NT) {
            const double wo = w[i];
            xh[i] = xh[i] + phi_rho * wo;
            if (la > 0.0) {
                const double vi = h[i] / la;
                v[i] = vi;
                Mv[i] = z[i] / la;
                w[i] = vi - theta_rho * wo;
            }
        }
        if (lstop) {
            done = 1;
            status = lstatus;
        }
    }

    // x = D x_hat; true ||A^T (b - A x)|| = ||D^{-1} A_hat^T (P b - A_hat x_hat)||
    __syncthreads();
    for (int i = tid; i < n; i += NT) xo[i] = xh[i] / colnorm[i];
    wg_spmv<NT, GS>(d.A, d.xh, d.q, red);
    __syncthreads();
    for (int i = tid; i < m; i += NT) r[i] = bb[perm[i]] - q[i];
    __syncthreads();
    wg_spmv<NT, GS>(d.AT, d.r, d.z, red);
    __syncthreads();
    sq = 0.0;
    for (int i = tid; i < n; i += NT) {
        const double c = colnorm[i] * z[i];
        sq += c * c;
    }
    const double atr = sqrt(wg_sum<NT>(sq, red));
    if (tid == 0) {
        d.out->atr = atr;
        d.out->nb = nb;
        d.out->iters = iter;
        d.out->status = status;
    }
}

// ------------------------------------------------------------------ compiled tiles

// Kernels of one tile: [precision FP64 / FP32].
struct TileEntry {
    rsilu_tile_t tile;
    const void *fn[2];
};

template <int NT, int GS, int GT>
TileEntry tile_entry()
{
    TileEntry e{{NT, GS, GT, 0}, {}};
    e.fn[0] = reinterpret_cast<const void *>(&k_batch_lsqr<double, NT, GS, GT>);
    e.fn[1] = reinterpret_cast<const void *>(&k_batch_lsqr<float, NT, GS, GT>);
    return e;
}

// Dynamic LDS of a launch for the triangular-solve vectors: 2 n values of its
// largest problem that fits in this bound; problems above it use global memory.
// A 1024-thread workgroup has its compute unit to itself and takes most of the
// 160 KiB; smaller workgroups keep 64 KiB so that several share a compute unit.
constexpr size_t xl_bound(int32_t threads) { return threads >= 1024 ? 144 * 1024 : 64 * 1024; }

const std::vector<TileEntry> &tiles()
{
    static const std::vector<TileEntry> t = {
        tile_entry<256, 4, 1>(),  tile_entry<256, 4, 4>(),  tile_entry<256, 8, 1>(),  tile_entry<256, 8, 4>(),
        tile_entry<512, 4, 1>(),  tile_entry<512, 4, 4>(),  tile_entry<512, 8, 1>(),  tile_entry<512, 8, 4>(),
        tile_entry<1024, 4, 1>(), tile_entry<1024, 4, 4>(), tile_entry<1024, 8, 1>(), tile_entry<1024, 8, 4>(),
    };
    return t;
}

const TileEntry *find_tile(const rsilu_tile_t &t)
{
    for (const TileEntry &e : tiles())
        if (e.tile.threads == t.threads && e.tile.spmv_lanes == t.spmv_lanes && e.tile.tri_lanes == t.tri_lanes &&
            t.reserved == 0)
            return &e;
    return nullptr;
}

constexpr rsilu_tile_t kDefaultTile = {1024, 4, 4, 0};

// ------------------------------------------------------------------ fixed descriptor table

// rsilu_batch_solve_static: the descriptor table and outcome slots of one launch in a
// fixed device array (one copy per GPU, for the process lifetime), so that the call
// allocates nothing. In host code `scratch` is only a handle for the symbol: its device
// address on each GPU comes from hipGetSymbolAddress, with that GPU current.
constexpr int32_t kStaticBatchMax = 256;
constexpr size_t kStaticDescBytes = ((sizeof(BDesc) * kStaticBatchMax + 255) / 256) * 256;
constexpr size_t kStaticBytes = kStaticDescBytes + sizeof(BOut) * kStaticBatchMax;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// ------------------------------------------------------------------ host side

template <class T>
T *at(const Ctx &c, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(c.dev) + off);
}

BOp bop(const Ctx &c, const DevCsrOff &o, const DevPlanOff &p)
{
    return BOp{at<int32_t>(c, o.ptr), at<int32_t>(c, o.col), at<void>(c, o.val), at<int32_t>(c, p.long_rows),
               o.nrows, p.nlong, p.long_thresh, 0};
}

// The M_b correction the batched kernel applies: 0 none (no A2 rows, or S^ absent),
// 1 Chebyshev steps through the explicit Y~; -1 a correction it does not implement.
int32_t correction_of(const Ctx &c)
{
    if (c.L2.nrows == 0 || c.smode == RSILU_S_NONE) return 0;
    return c.smode == RSILU_S_CHEB && yexplicit(c) ? 1 : -1;
}

BTri btri(const Ctx &c, const DevTriOff &o)
{
    return BTri{at<int32_t>(c, o.lev), at<int32_t>(c, o.rows), at<int32_t>(c, o.lo.ptr), at<int32_t>(c, o.lo.col),
                at<void>(c, o.lo.val), o.ldiag ? at<void>(c, o.ldiag) : nullptr, at<void>(c, o.lrec), o.nlev, 0};
}

// Whether the batched kernel takes a handle's configuration.
rsilu_status_t check_config(const Ctx &c)
{
    if (c.prm.krylov != RSILU_KRYLOV_LSQR || c.prm.form != RSILU_FORM_ALG2) return RSILU_EINVAL;
    if (correction_of(c) < 0) return RSILU_EINVAL;
    if (c.R.nrows > 0) return RSILU_EINVAL;  // removed rows change the preconditioner
    return RSILU_OK;
}

// Whether a handle can be solved by the batched kernel.
rsilu_status_t check_handle(const Ctx &c)
{
    if (!c.dev) return RSILU_EINVAL;
    return check_config(c);
}

BDesc make_desc(const Ctx &c, const double *b, double *x, double tol, int32_t maxit, BOut *out)
{
    const Layout &L = c.lay;
    BDesc d;
    std::memset(&d, 0, sizeof(d));
    d.A = bop(c, L.A, L.pA);
    d.AT = bop(c, L.AT, L.pAT);
    d.tri[0] = btri(c, L.UTf);
    d.tri[1] = btri(c, L.L1b);
    d.tri[2] = btri(c, L.L1f);
    d.tri[3] = btri(c, L.Ub);
    d.perm = at<int32_t>(c, L.perm);
    d.colnorm = at<double>(c, L.colnorm);
    d.b = b;
    d.x = x;
    d.xh = at<double>(c, L.xh);
    d.z = at<double>(c, L.z);
    d.h = at<double>(c, L.h);
    d.r = at<double>(c, L.r);
    d.q = at<double>(c, L.q);
    d.v = at<double>(c, L.l_v);
    d.Mv = at<double>(c, L.l_mv);
    d.w = at<double>(c, L.l_w);
    // preconditioner vectors: the same buffers as the multi-kernel path's Algorithm 2
    d.pt0 = at<void>(c, L.t);
    d.pt1 = at<void>(c, L.gp);
    d.pt2 = at<void>(c, L.v);
    if (fp32(c)) {
        d.pin = at<void>(c, L.f32a);
        d.pout = at<void>(c, L.f32b);
    }
    d.corr = correction_of(c);
    d.k = (int32_t)c.L2.nrows;
    if (d.corr > 0) {
        d.Y = bop(c, L.Y, L.pY);
        d.YT = bop(c, L.YT, L.pYT);
        d.cg = at<void>(c, L.s2);
        d.cy = at<void>(c, L.y);
        d.ct = at<void>(c, L.c2);
        d.cu = at<void>(c, L.u);
        d.cheb = at<double>(c, L.cheb);
        d.cheb_theta = c.cheb_theta;
        d.cheb_omega = c.cheb_omega;
        d.cheb_K = c.cheb_K;
        d.cr = at<void>(c, L.cg_r);
        d.cd = at<void>(c, L.cg_p);
        d.cw = at<void>(c, L.cg_w);
        d.cq = at<void>(c, L.cg_q);
    }
    d.tol = tol;
    d.maxit = maxit;
    d.m = (int32_t)c.m;
    d.n = (int32_t)c.n;
    d.out = out;
    return d;
}

// Rough work of one problem (entries streamed per iteration plus the levels,
// which cost a barrier each): problems are ordered by it, largest first, so the
// longest workgroups start first.
double work_of(const Ctx &c)
{
    const int32_t corr = correction_of(c);
    const double ny = corr > 0 ? (double)c.Yd.nnz() * (2.0 + 2.0 * c.cheb_K) : 0.0;
    return 2.0 * (double)c.nnz_a + (double)(c.L1.nnz() * 2 + c.U.nnz() * 2) + ny +
           2000.0 * (double)(c.lvL1.nlev() * 2 + c.lvU.nlev() + c.lvUT.nlev());
}

rsilu_status_t map_status(const BOut &o, int32_t maxit)
{
    if (o.status == 2) return RSILU_BREAKDOWN;
    if (maxit == 0 && o.nb > 0.0) return RSILU_NOT_CONVERGED;
    if (o.status == 1) return RSILU_NOT_CONVERGED;
    return RSILU_OK;
}

}  // namespace
}  // namespace rsilu

using namespace rsilu;

struct rsilu_batch {
    int32_t cap = 0;
    int device = -1;
    BDesc *d_desc = nullptr;
    BOut *d_out = nullptr;
    BDesc *h_desc = nullptr;  // pinned
    BOut *h_out = nullptr;    // pinned
    hipStream_t cap_stream = nullptr;
    hipStream_t aux_stream = nullptr;  // plain-path solves of rsilu_batch_solve_auto
    hipEvent_t ev_in = nullptr;        // the caller's stream up to the call (aux_stream waits on it)
    hipEvent_t ev_out = nullptr;       // aux_stream's plain solves (the caller's stream waits on it)
    std::map<std::tuple<int32_t, const void *, size_t>, hipGraphExec_t> graphs;  // (count, kernel, LDS)
    std::mutex mu;  // one launch at a time per batch object
};

namespace rsilu {
namespace {

#define RSILU_HIPB(call)                               \
    do {                                               \
        if ((call) != hipSuccess) return RSILU_EHIP;   \
    } while (0)

// Descriptor upload, kernel, outcome download: enqueued directly, or captured
// once per (count, kernel, dynamic LDS) and replayed.
rsilu_status_t run_batch(rsilu_batch &bt, int32_t count, const void *fn, int32_t threads, size_t shmem,
                         bool use_graph, hipStream_t s, const std::function<void()> &during)
{
    const size_t db = sizeof(BDesc) * (size_t)count, ob = sizeof(BOut) * (size_t)count;
    auto enqueue = [&](hipStream_t st) -> hipError_t {
        hipError_t e = hipMemcpyAsync(bt.d_desc, bt.h_desc, db, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        BDesc *arg = bt.d_desc;
        uint32_t xlb = (uint32_t)shmem;
        void *args[] = {&arg, &xlb};
        e = hipLaunchKernel(fn, dim3((unsigned)count), dim3((unsigned)threads), args, shmem, st);
        if (e != hipSuccess) return e;
        return hipMemcpyAsync(bt.h_out, bt.d_out, ob, hipMemcpyDeviceToHost, st);
    };
    if (!use_graph) {
        RSILU_HIPB(enqueue(s));
        if (during) during();
        RSILU_HIPB(hipStreamSynchronize(s));
        return RSILU_OK;
    }
    const auto key = std::make_tuple(count, fn, shmem);
    auto it = bt.graphs.find(key);
    if (it == bt.graphs.end()) {
        if (!bt.cap_stream) RSILU_HIPB(hipStreamCreateWithFlags(&bt.cap_stream, hipStreamNonBlocking));
        RSILU_HIPB(hipStreamBeginCapture(bt.cap_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t ce = enqueue(bt.cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(bt.cap_stream, &g);
        if (ce != hipSuccess || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return RSILU_EHIP;
        }
        hipGraphExec_t x = nullptr;
        const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return RSILU_EHIP;
        it = bt.graphs.emplace(key, x).first;
    }
    RSILU_HIPB(hipGraphLaunch(it->second, s));
    if (during) during();
    RSILU_HIPB(hipStreamSynchronize(s));
    return RSILU_OK;
}

// Batched solve with an optional maxit override (>= 0) used by the autotuner;
// `during` runs on the host while the first launch is on the device.
rsilu_status_t batch_solve(rsilu_batch &bt, int32_t count, const rsilu_handle_t *hs, const double *const *b,
                           const double *tol, double *const *x, const rsilu_tile_t *tile, rsilu_batch_result_t *res,
                           hipStream_t s, int32_t maxit_override, std::function<void()> during = nullptr)
{
    if (count < 0 || count > bt.cap) return RSILU_EINVAL;
    if (count == 0) return RSILU_OK;
    if (!hs || !b || !tol || !x || !res) return RSILU_EINVAL;
    const TileEntry *te = find_tile(tile ? *tile : kDefaultTile);
    if (!te) return RSILU_EINVAL;
    bool any32 = false, any64 = false;
    for (int32_t i = 0; i < count; ++i) {
        if (!hs[i] || !b[i] || !x[i] || static_cast<const void *>(b[i]) == static_cast<const void *>(x[i]))
            return RSILU_EINVAL;
        if (!(tol[i] >= 0.0) || !std::isfinite(tol[i])) return RSILU_EINVAL;
        const rsilu_status_t st = check_handle(*hs[i]);
        if (st != RSILU_OK) return st;
        if (hs[i]->device != bt.device) return RSILU_ESTATE;
        (fp32(*hs[i]) ? any32 : any64) = true;
        for (int32_t j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return RSILU_EINVAL;
    }
    // FP64 and FP32 preconditioners are different kernels: one launch each
    std::vector<int32_t> order((size_t)count);
    for (int32_t i = 0; i < count; ++i) order[i] = i;
    std::vector<double> work((size_t)count);
    for (int32_t i = 0; i < count; ++i) work[i] = work_of(*hs[i]);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return work[a] > work[c]; });
    std::lock_guard<std::mutex> lk(bt.mu);
    for (int pass = 0; pass < 2; ++pass) {
        const bool fp = pass == 1;
        if ((fp && !any32) || (!fp && !any64)) continue;
        std::vector<int32_t> idx;
        for (int32_t i : order)
            if (fp32(*hs[i]) == fp) idx.push_back(i);
        const int32_t k = (int32_t)idx.size();
        const size_t vb = fp ? sizeof(float) : sizeof(double);
        size_t xl = 0;
        for (int32_t j = 0; j < k; ++j) {
            const Ctx &c = *hs[idx[j]];
            const int32_t mi = maxit_override >= 0 ? maxit_override : c.prm.maxit;
            bt.h_desc[j] = make_desc(c, b[idx[j]], x[idx[j]], tol[idx[j]], mi, bt.d_out + j);
            const size_t need = 2 * (size_t)c.n * vb;
            if (need <= xl_bound(te->tile.threads)) xl = std::max(xl, need);
        }
        const rsilu_status_t rc =
            run_batch(bt, k, te->fn[fp ? 1 : 0], te->tile.threads, xl, maxit_override < 0, s, during);
        during = nullptr;
        if (rc != RSILU_OK) return rc;
        for (int32_t j = 0; j < k; ++j) {
            const BOut &o = bt.h_out[j];
            const Ctx &c = *hs[idx[j]];
            rsilu_batch_result_t &r = res[idx[j]];
            r.iters = o.iters;
            r.atr_norm = o.atr;
            r.atr_rel = o.nb > 0.0 ? o.atr / o.nb : 0.0;
            r.status = map_status(o, maxit_override >= 0 ? maxit_override : c.prm.maxit);
        }
    }
    return RSILU_OK;
}

}  // namespace
}  // namespace rsilu

// ------------------------------------------------------------------ autotuner

struct rsilu_tuner {
    double slack = 1.0;
    int32_t iters = 8;
    rsilu_batch_t bt = nullptr;  // single-problem batch object for timing
    std::map<std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t>, rsilu_tune_result_t> cache;
    std::mutex mu;
};

namespace rsilu {
namespace {

int32_t log2_class(double v) { return v <= 1.0 ? 0 : (int32_t)std::floor(std::log2(v)); }

// Signature of a problem: precision, size class, density class, level class,
// whether long rows are present, and the correction's class (none, or the
// products with Y~ per application relative to those with A_hat).
std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t> signature(const Ctx &c)
{
    const double nnz_per_row = c.m ? (double)c.nnz_a / (double)c.m : 0.0;
    const int32_t levels = c.lvL1.nlev() + c.lvL1T.nlev() + c.lvU.nlev() + c.lvUT.nlev();
    const int32_t corr = correction_of(c);
    const double yrel =
        corr > 0 ? (double)c.Yd.nnz() * (2.0 + 2.0 * c.cheb_K) / std::max(1.0, 2.0 * (double)c.nnz_a) : 0.0;
    return std::make_tuple((int32_t)fp32(c), log2_class((double)c.n), log2_class(4.0 * nnz_per_row),
                           log2_class((double)levels), (int32_t)(c.plA.long_rows.size() > 0),
                           corr > 0 ? 1 + log2_class(2.0 * yrel) : 0);
}

double elapsed_ms(std::chrono::steady_clock::time_point a)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
}

}  // namespace
}  // namespace rsilu

extern "C" {

int32_t rsilu_batch_accepts(rsilu_handle_t h) { return h && check_config(*h) == RSILU_OK ? 1 : 0; }

int32_t rsilu_batch_tiles(rsilu_tile_t *out, int32_t max)
{
    const auto &t = tiles();
    if (out)
        for (int32_t i = 0; i < max && i < (int32_t)t.size(); ++i) out[i] = t[(size_t)i].tile;
    return (int32_t)t.size();
}

rsilu_status_t rsilu_batch_create(int32_t capacity, rsilu_batch_t *out)
{
    if (!out || capacity < 1 || capacity > 65535) return RSILU_EINVAL;
    *out = nullptr;
    rsilu_batch *bt = nullptr;
    try {
        bt = new rsilu_batch();
    } catch (const std::bad_alloc &) {
        return RSILU_ENOMEM;
    }
    bt->cap = capacity;
    if (hipGetDevice(&bt->device) != hipSuccess) {
        delete bt;
        return RSILU_EHIP;
    }
    const size_t db = sizeof(BDesc) * (size_t)capacity, ob = sizeof(BOut) * (size_t)capacity;
    if (hipMalloc(&bt->d_desc, db) != hipSuccess || hipMalloc(&bt->d_out, ob) != hipSuccess ||
        hipHostMalloc(&bt->h_desc, db, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&bt->h_out, ob, hipHostMallocDefault) != hipSuccess) {
        rsilu_batch_destroy(bt);
        return RSILU_ENOMEM;
    }
    std::memset(bt->h_desc, 0, db);
    std::memset(bt->h_out, 0, ob);
    *out = bt;
    return RSILU_OK;
}

rsilu_status_t rsilu_batch_solve(rsilu_batch_t bt, int32_t count, const rsilu_handle_t *hs, const double *const *b,
                                 const double *tol, double *const *x, const rsilu_tile_t *tile,
                                 rsilu_batch_result_t *res, hipStream_t s)
{
    if (!bt) return RSILU_EINVAL;
    try {
        return batch_solve(*bt, count, hs, b, tol, x, tile, res, s, -1);
    } catch (const std::bad_alloc &) {
        return RSILU_ENOMEM;
    }
}

void rsilu_batch_destroy(rsilu_batch_t bt)
{
    if (!bt) return;
    for (auto &kv : bt->graphs) (void)hipGraphExecDestroy(kv.second);
    if (bt->cap_stream) (void)hipStreamDestroy(bt->cap_stream);
    if (bt->aux_stream) (void)hipStreamDestroy(bt->aux_stream);
    if (bt->ev_in) (void)hipEventDestroy(bt->ev_in);
    if (bt->ev_out) (void)hipEventDestroy(bt->ev_out);
    if (bt->d_desc) (void)hipFree(bt->d_desc);
    if (bt->d_out) (void)hipFree(bt->d_out);
    if (bt->h_desc) (void)hipHostFree(bt->h_desc);
    if (bt->h_out) (void)hipHostFree(bt->h_out);
    delete bt;
}

}  // extern "C"

namespace {

constexpr int kStaticDevices = 64;

struct StaticBatchState {
    std::mutex mu;                      // one call at a time in this process
    unsigned char *dev[kStaticDevices] = {};  // device address of `scratch` per GPU
    BDesc h_desc[kStaticBatchMax];      // host staging (pageable; the copies are synchronised)
    BOut h_out[kStaticBatchMax];
};

StaticBatchState &static_state()
{
    static StaticBatchState st;
    return st;
}

}  // namespace

extern "C" {

rsilu_status_t rsilu_batch_solve_static(int32_t count, const rsilu_handle_t *hs, const double *const *b,
                                        const double *tol, double *const *x, const rsilu_tile_t *tile,
                                        rsilu_batch_result_t *res, hipStream_t s)
{
    if (count < 0 || count > kStaticBatchMax) return RSILU_EINVAL;
    if (count == 0) return RSILU_OK;
    if (!hs || !b || !tol || !x || !res) return RSILU_EINVAL;
    const TileEntry *te = find_tile(tile ? *tile : kDefaultTile);
    if (!te) return RSILU_EINVAL;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) return RSILU_EHIP;
    if (device < 0 || device >= kStaticDevices) return RSILU_EINVAL;
    bool any32 = false, any64 = false;
    for (int32_t i = 0; i < count; ++i) {
        if (!hs[i] || !b[i] || !x[i] || static_cast<const void *>(b[i]) == static_cast<const void *>(x[i]))
            return RSILU_EINVAL;
        if (!(tol[i] >= 0.0) || !std::isfinite(tol[i])) return RSILU_EINVAL;
        const rsilu_status_t st = check_handle(*hs[i]);
        if (st != RSILU_OK) return st;
        if (hs[i]->device != device) return RSILU_ESTATE;
        (fp32(*hs[i]) ? any32 : any64) = true;
        for (int32_t j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return RSILU_EINVAL;
    }
    StaticBatchState &S = static_state();
    std::lock_guard<std::mutex> lk(S.mu);
    if (!S.dev[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RSILU_EHIP;
        S.dev[device] = static_cast<unsigned char *>(p);
    }
    BDesc *d_desc = reinterpret_cast<BDesc *>(S.dev[device]);
    BOut *d_out = reinterpret_cast<BOut *>(S.dev[device] + kStaticDescBytes);
    // largest problems first, as rsilu_batch_solve orders them (insertion sort: no allocation)
    int32_t order[kStaticBatchMax];
    for (int32_t i = 0; i < count; ++i) {
        const double wi = work_of(*hs[i]);
        int32_t j = i;
        while (j > 0 && work_of(*hs[order[j - 1]]) < wi) {
            order[j] = order[j - 1];
            --j;
        }
        order[j] = i;
    }
    for (int pass = 0; pass < 2; ++pass) {
        const bool fp = pass == 1;
        if ((fp && !any32) || (!fp && !any64)) continue;
        int32_t idx[kStaticBatchMax];
        int32_t k = 0;
        for (int32_t t = 0; t < count; ++t)
            if (fp32(*hs[order[t]]) == fp) idx[k++] = order[t];
        const size_t vb = fp ? sizeof(float) : sizeof(double);
        size_t xl = 0;
        for (int32_t j = 0; j < k; ++j) {
            const Ctx &c = *hs[idx[j]];
            S.h_desc[j] = make_desc(c, b[idx[j]], x[idx[j]], tol[idx[j]], c.prm.maxit, d_out + j);
            const size_t need = 2 * (size_t)c.n * vb;
            if (need <= xl_bound(te->tile.threads)) xl = std::max(xl, need);
        }
        if (hipMemcpyAsync(d_desc, S.h_desc, sizeof(BDesc) * (size_t)k, hipMemcpyHostToDevice, s) != hipSuccess)
            return RSILU_EHIP;
        BDesc *arg = d_desc;
        uint32_t xlb = (uint32_t)xl;
        void *args[] = {&arg, &xlb};
        if (hipLaunchKernel(te->fn[fp ? 1 : 0], dim3((unsigned)k), dim3((unsigned)te->tile.threads), args, xl, s) !=
            hipSuccess)
            return RSILU_EHIP;
        if (hipMemcpyAsync(S.h_out, d_out, sizeof(BOut) * (size_t)k, hipMemcpyDeviceToHost, s) != hipSuccess)
            return RSILU_EHIP;
        if (hipStreamSynchronize(s) != hipSuccess) return RSILU_EHIP;
        for (int32_t j = 0; j < k; ++j) {
            const BOut &o = S.h_out[j];
            rsilu_batch_result_t &r = res[idx[j]];
            r.iters = o.iters;
            r.atr_norm = o.atr;
            r.atr_rel = o.nb > 0.0 ? o.atr / o.nb : 0.0;
            r.status = map_status(o, hs[idx[j]]->prm.maxit);
        }
    }
    return RSILU_OK;
}

int32_t rsilu_batch_static_max(void) { return kStaticBatchMax; }

rsilu_status_t rsilu_tuner_create(double slack, int32_t iters, rsilu_tuner_t *out)
{
    if (!out || !std::isfinite(slack) || !(slack > 0.0) || iters < 2) return RSILU_EINVAL;
    *out = nullptr;
    rsilu_tuner *t = nullptr;
    try {
        t = new rsilu_tuner();
    } catch (const std::bad_alloc &) {
        return RSILU_ENOMEM;
    }
    t->slack = slack;
    t->iters = iters;
    const rsilu_status_t rc = rsilu_batch_create(1, &t->bt);
    if (rc != RSILU_OK) {
        delete t;
        return rc;
    }
    *out = t;
    return RSILU_OK;
}

rsilu_status_t rsilu_tune(rsilu_tuner_t t, rsilu_handle_t h, const double *b_dev, double *x_dev,
                          rsilu_tune_result_t *res, hipStream_t s)
{
    if (!t || !h || !b_dev || !x_dev || !res) return RSILU_EINVAL;
    rsilu_status_t rc = check_handle(*h);
    if (rc != RSILU_OK) return rc;
    std::lock_guard<std::mutex> lk(t->mu);
    const auto key = signature(*h);
    auto it = t->cache.find(key);
    if (it != t->cache.end()) {
        *res = it->second;
        res->from_cache = 1;
        return RSILU_OK;
    }
    const int32_t K = std::min<int32_t>(t->iters, std::max<int32_t>(h->prm.maxit, 2));
    const double zero = 0.0;
    rsilu_batch_result_t br;
    // the plain path first: one untimed run (first touch of the problem's data), one
    // timed run, with the same iteration count
    const int32_t saved = h->prm.maxit;
    h->prm.maxit = K;
    double plain = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
        const auto t0 = std::chrono::steady_clock::now();
        int32_t it_ = 0;
        double a = 0.0, ar = 0.0;
        rc = rsilu_solve(h, b_dev, 0.0, x_dev, &it_, &a, &ar, s);
        if (rc < 0) break;
        if (rep == 1) plain = elapsed_ms(t0);
    }
    h->prm.maxit = saved;
    if (rc < 0) return rc;
    // the batched kernel: the default tile, and every other compiled tile only when the
    // default one is within twice the slack of the plain path (a problem far too large
    // for one workgroup is not timed twelve times)
    double best = 1e300;
    rsilu_tile_t best_tile = kDefaultTile;
    for (int pass = 0; pass < 2; ++pass) {
        for (const TileEntry &e : tiles()) {
            const bool dflt = std::memcmp(&e.tile, &kDefaultTile, sizeof(rsilu_tile_t)) == 0;
            if (dflt != (pass == 0)) continue;
            const auto t0 = std::chrono::steady_clock::now();
            rc = batch_solve(*t->bt, 1, &h, &b_dev, &zero, &x_dev, &e.tile, &br, s, K);
            if (rc != RSILU_OK) return rc;
            const double ms = elapsed_ms(t0);
            if (ms < best) {
                best = ms;
                best_tile = e.tile;
            }
        }
        if (best > 2.0 * t->slack * plain) break;
    }
    rsilu_tune_result_t r{};
    r.tile = best_tile;
    r.batched_ms_per_iter = best / K;
    r.plain_ms_per_iter = plain / K;
    r.path = best <= t->slack * plain ? 0 : 1;
    r.from_cache = 0;
    t->cache.emplace(key, r);
    *res = r;
    return RSILU_OK;
}

rsilu_status_t rsilu_batch_solve_auto(rsilu_batch_t bt, rsilu_tuner_t t, int32_t count, const rsilu_handle_t *hs,
                                      const double *const *b, const double *tol, double *const *x,
                                      rsilu_batch_result_t *res, int32_t *path, rsilu_tile_t *tile_used,
                                      hipStream_t s)
{
    if (!bt || !t || count < 0 || count > bt->cap) return RSILU_EINVAL;
    if (count == 0) return RSILU_OK;
    if (!hs || !b || !tol || !x || !res || !path) return RSILU_EINVAL;
    for (int32_t i = 0; i < count; ++i) {
        if (!hs[i] || !b[i] || !x[i] || static_cast<const void *>(b[i]) == static_cast<const void *>(x[i]) ||
            !hs[i]->dev)
            return RSILU_EINVAL;
        if (!(tol[i] >= 0.0) || !std::isfinite(tol[i])) return RSILU_EINVAL;
        for (int32_t j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return RSILU_EINVAL;
    }
    try {
        // times per iteration of every accepted problem (cached per signature)
        std::vector<rsilu_tune_result_t> tr((size_t)count);
        std::vector<int32_t> acc, tuned_plain;
        for (int32_t i = 0; i < count; ++i) {
            path[i] = 1;
            if (check_handle(*hs[i]) != RSILU_OK) continue;
            const rsilu_status_t rc = rsilu_tune(t, hs[i], b[i], x[i], &tr[(size_t)i], s);
            if (rc != RSILU_OK) return rc;
            (tr[(size_t)i].path == 0 ? acc : tuned_plain).push_back(i);
        }
        // The problems the tuner gives to the batched kernel start on the batched launch,
        // which lasts as long as its slowest problem; the plain path runs the others one
        // after another beside it. Move the slowest batched problem to the plain path while
        // that shortens max(slowest batched, sum of plain) (equal iteration counts assumed).
        std::stable_sort(acc.begin(), acc.end(), [&](int32_t a, int32_t c) {
            return tr[(size_t)a].batched_ms_per_iter > tr[(size_t)c].batched_ms_per_iter;
        });
        double sum_p = 0.0;
        for (int32_t i : tuned_plain) sum_p += tr[(size_t)i].plain_ms_per_iter;
        size_t top = 0;
        while (top < acc.size()) {
            const rsilu_tune_result_t &r = tr[(size_t)acc[top]];
            const double now = std::max(r.batched_ms_per_iter, sum_p);
            const double next_b = top + 1 < acc.size() ? tr[(size_t)acc[top + 1]].batched_ms_per_iter : 0.0;
            if (std::max(next_b, sum_p + r.plain_ms_per_iter) >= now) break;
            sum_p += r.plain_ms_per_iter;
            ++top;
        }
        std::vector<int32_t> plain;
        for (int32_t i = 0; i < count; ++i)
            if (check_handle(*hs[i]) != RSILU_OK) plain.push_back(i);
        for (int32_t i : tuned_plain) plain.push_back(i);
        for (size_t q = 0; q < top; ++q) plain.push_back(acc[q]);
        std::vector<int32_t> batched(acc.begin() + (ptrdiff_t)top, acc.end());
        // one tile for the launch: the tuned tile of its slowest problem
        rsilu_tile_t tile = batched.empty() ? kDefaultTile : tr[(size_t)batched.front()].tile;
        if (tile_used) *tile_used = tile;
        rsilu_status_t plain_rc = RSILU_OK;
        auto run_plain = [&](hipStream_t ps) {
            for (int32_t i : plain) {
                rsilu_batch_result_t &r = res[i];
                const rsilu_status_t rc = rsilu_solve(hs[i], b[i], tol[i], x[i], &r.iters, &r.atr_norm, &r.atr_rel, ps);
                r.status = rc;
                if (rc < 0) plain_rc = rc;
            }
        };
        if (batched.empty()) {
            run_plain(s);
            return plain_rc;
        }
        if (!plain.empty()) {
            if (!bt->aux_stream && hipStreamCreateWithFlags(&bt->aux_stream, hipStreamNonBlocking) != hipSuccess)
                return RSILU_EHIP;
            if (!bt->ev_in && hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming) != hipSuccess)
                return RSILU_EHIP;
            if (!bt->ev_out && hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming) != hipSuccess)
                return RSILU_EHIP;
            // the plain solves on aux_stream start after the work the caller queued on s
            // (copies of b, for instance), and s resumes only after them
            if (hipEventRecord(bt->ev_in, s) != hipSuccess || hipStreamWaitEvent(bt->aux_stream, bt->ev_in, 0) != hipSuccess)
                return RSILU_EHIP;
        }
        std::vector<rsilu_handle_t> bh;
        std::vector<const double *> bb;
        std::vector<double> bt_tol;
        std::vector<double *> bx;
        for (int32_t i : batched) {
            path[i] = 0;
            bh.push_back(hs[i]);
            bb.push_back(b[i]);
            bt_tol.push_back(tol[i]);
            bx.push_back(x[i]);
        }
        std::vector<rsilu_batch_result_t> br(batched.size());
        const rsilu_status_t rc =
            batch_solve(*bt, (int32_t)batched.size(), bh.data(), bb.data(), bt_tol.data(), bx.data(), &tile, br.data(),
                        s, -1, plain.empty() ? std::function<void()>() : std::function<void()>([&] { run_plain(bt->aux_stream); }));
        if (!plain.empty() &&
            (hipEventRecord(bt->ev_out, bt->aux_stream) != hipSuccess || hipStreamWaitEvent(s, bt->ev_out, 0) != hipSuccess))
            return RSILU_EHIP;
        if (rc != RSILU_OK) return rc;
        for (size_t q = 0; q < batched.size(); ++q) res[batched[q]] = br[q];
        return plain_rc;
    } catch (const std::bad_alloc &) {
        return RSILU_ENOMEM;
    }
}

int32_t rsilu_tuner_size(rsilu_tuner_t t)
{
    if (!t) return 0;
    std::lock_guard<std::mutex> lk(t->mu);
    return (int32_t)t->cache.size();
}

void rsilu_tuner_destroy(rsilu_tuner_t t)
{
    if (!t) return;
    rsilu_batch_destroy(t->bt);
    delete t;
}

}  // extern "C"
