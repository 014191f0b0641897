// C ABI of the library and the device driver of the solve (Algorithm 1 with
// Algorithm 3 or Algorithm 2), enqueued on the caller's stream. The host only enqueues work
// and polls a stop flag every `poll` iterations; every scalar of the
// recurrence lives on the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <type_traits>

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "kernels.hpp"

namespace rsilu {
namespace {

struct PinnedMail {
    DevState init;  // host -> device at the start of a solve
    DevState poll;  // device -> host while polling
};

#define RSILU_HIP(call)                                \
    do {                                               \
        if ((call) != hipSuccess) return RSILU_EHIP;   \
    } while (0)

template <class T>
T *at(const Ctx &c, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(c.dev) + off);
}

DCsr dcsr(const Ctx &c, const DevCsrOff &o)
{
    return DCsr{at<int32_t>(c, o.ptr), at<int32_t>(c, o.col), at<double>(c, o.val), o.nrows};
}

DPlan dplan(const Ctx &c, const DevPlanOff &o)
{
    return DPlan{at<int32_t>(c, o.long_rows), at<int32_t>(c, o.seg_ptr), at<int32_t>(c, o.seg_beg),
                 at<int32_t>(c, o.seg_end), o.nlong, o.nseg, o.lanes, o.long_thresh, o.unroll};
}

DTri dtri(const Ctx &c, const DevTriOff &o)
{
    return DTri{dcsr(c, o.a), o.diag ? at<double>(c, o.diag) : nullptr, at<int32_t>(c, o.rows),
                at<int32_t>(c, o.chunk), o.nchunks, o.lanes};
}

// HIP events around one launch group of a profiled class (rsilu_set_profiling).
class ProfScope {
public:
    ProfScope(Ctx &c, hipStream_t s, int cls, double bytes = 0.0) : c_(c), s_(s), cls_(cls), bytes_(bytes)
    {
        if (!c_.prof || !((c_.prof_mask >> cls_) & 1u)) return;
        while (c_.ev_next + 2 > c_.ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            c_.ev_pool.push_back(static_cast<void *>(e));
        }
        idx_ = (int)c_.ev_next;
        if (hipEventRecord(static_cast<hipEvent_t>(c_.ev_pool[(size_t)idx_]), s_) != hipSuccess) {
            idx_ = -1;
            return;
        }
        c_.ev_next += 2;
    }
    ~ProfScope()
    {
        if (idx_ < 0) return;
        if (hipEventRecord(static_cast<hipEvent_t>(c_.ev_pool[(size_t)idx_ + 1]), s_) == hipSuccess)
            c_.ev_open.push_back({cls_, idx_, c_.ev_iter, bytes_});
    }

private:
    Ctx &c_;
    hipStream_t s_;
    int cls_;
    double bytes_;
    int idx_ = -1;
};

// After a stream synchronisation: add up the recorded launches of the
// iterations that really ran (later ones returned at once on the stop flag).
void prof_collect(Ctx &c, int completed_iters)
{
    for (const Ctx::EvRec &r : c.ev_open) {
        if (r.iter > completed_iters) continue;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, static_cast<hipEvent_t>(c.ev_pool[(size_t)r.idx]),
                                static_cast<hipEvent_t>(c.ev_pool[(size_t)r.idx + 1])) == hipSuccess) {
            c.prof_ms[r.cls] += ms;
            c.prof_launches[r.cls] += 1;
            c.prof_bytes[r.cls] += r.bytes;
        }
    }
    c.ev_open.clear();
    c.ev_next = 0;
}

// Device pointers of one solve.
struct Ptrs {
    DevState *st;
    const int32_t *done;
    double *partials, *segpart;
    DCsr A, AT, L2, L2T;
    DPlan pA, pAT, pL2, pL2T, pY, pYT;
    DTri L1f, L1b, Ub, UTf;
    const int32_t *perm;
    const double *colnorm, *sfac;
    double *xh, *p, *z, *h, *t, *y, *v, *g, *gp, *s2, *c2, *r, *q, *u;
    double *lo_rhs, *lo_add;
};

Ptrs ptrs(const Ctx &c)
{
    const Layout &L = c.lay;
    Ptrs P;
    P.st = at<DevState>(c, L.state);
    P.done = &P.st->done;
    P.partials = at<double>(c, L.partials);
    P.segpart = at<double>(c, L.segpart);
    P.A = dcsr(c, L.A);
    P.AT = dcsr(c, L.AT);
    P.L2 = dcsr(c, L.L2);
    P.L2T = dcsr(c, L.L2T);
    P.pA = dplan(c, L.pA);
    P.pAT = dplan(c, L.pAT);
    P.pL2 = dplan(c, L.pL2);
    P.pL2T = dplan(c, L.pL2T);
    P.pY = dplan(c, L.pY);
    P.pYT = dplan(c, L.pYT);
    P.L1f = dtri(c, L.L1f);
    P.L1b = dtri(c, L.L1b);
    P.Ub = dtri(c, L.Ub);
    P.UTf = dtri(c, L.UTf);
    P.perm = at<int32_t>(c, L.perm);
    P.colnorm = at<double>(c, L.colnorm);
    P.sfac = at<double>(c, L.sfac);
    P.xh = at<double>(c, L.xh);
    P.p = at<double>(c, L.p);
    P.z = at<double>(c, L.z);
    P.h = at<double>(c, L.h);
    P.t = at<double>(c, L.t);
    P.y = at<double>(c, L.y);
    P.v = at<double>(c, L.v);
    P.g = at<double>(c, L.g);
    P.gp = at<double>(c, L.gp);
    P.s2 = at<double>(c, L.s2);
    P.c2 = at<double>(c, L.c2);
    P.r = at<double>(c, L.r);
    P.q = at<double>(c, L.q);
    P.u = at<double>(c, L.u);
    P.lo_rhs = at<double>(c, L.lo_rhs);
    P.lo_add = at<double>(c, L.lo_add);
    return P;
}

// Operators and work vectors of the preconditioner in its precision T
// (double, or float for the FP32 preconditioner: the factor operators then
// hold FP32 values and the work vectors are read as float arrays).
template <class T>
struct Pre {
    DCsrT<T> L2, L2T, Y, YT;  // Y, YT: the explicit Y~ (RSILU_Y_EXPLICIT)
    DTriT<T> L1f, L1b, Ub, UTf;
    T *t, *gp, *v, *g, *y, *s2, *c2, *u, *lo_rhs, *lo_add, *segpart;
};

template <class T>
DCsrT<T> dcsr_t(const Ctx &c, const DevCsrOff &o)
{
    return DCsrT<T>{at<int32_t>(c, o.ptr), at<int32_t>(c, o.col), at<T>(c, o.val), o.nrows};
}

template <class T>
DTriT<T> dtri_t(const Ctx &c, const DevTriOff &o)
{
    return DTriT<T>{dcsr_t<T>(c, o.a), o.diag ? at<T>(c, o.diag) : nullptr, at<int32_t>(c, o.rows),
                    at<int32_t>(c, o.chunk), o.nchunks, o.lanes};
}

template <class T>
Pre<T> pre(const Ctx &c)
{
    const Layout &L = c.lay;
    Pre<T> W;
    W.L2 = dcsr_t<T>(c, L.L2);
    W.L2T = dcsr_t<T>(c, L.L2T);
    W.Y = dcsr_t<T>(c, L.Y);
    W.YT = dcsr_t<T>(c, L.YT);
    W.L1f = dtri_t<T>(c, L.L1f);
    W.L1b = dtri_t<T>(c, L.L1b);
    W.Ub = dtri_t<T>(c, L.Ub);
    W.UTf = dtri_t<T>(c, L.UTf);
    W.t = at<T>(c, L.t);
    W.gp = at<T>(c, L.gp);
    W.v = at<T>(c, L.v);
    W.g = at<T>(c, L.g);
    W.y = at<T>(c, L.y);
    W.s2 = at<T>(c, L.s2);
    W.c2 = at<T>(c, L.c2);
    W.u = at<T>(c, L.u);
    W.lo_rhs = at<T>(c, L.lo_rhs);
    W.lo_add = at<T>(c, L.lo_add);
    W.segpart = at<T>(c, L.segpart);
    return W;
}

bool syncfree(const Ctx &c) { return c.prm.trsv == RSILU_TRSV_SYNCFREE; }

// One triangular solve with the configured schedule. Sync-free solves (FP64
// only) need x sentinel-filled and their ticket cleared beforehand.
template <class T>
void trsv(Ctx &c, hipStream_t s, const Ptrs &P, const Pre<T> &W, const DTriT<T> &t, const Levels &lv,
          const Sweep &sw, const DevTriOff &o, const T *rhs, T *x, const T *add, T *y2, int ticket,
          const int32_t *done, int cls)
{
    ProfScope ps(c, s, cls);
    if (c.prm.trsv == RSILU_TRSV_HYBRID) {
        const unsigned char *blob = at<unsigned char>(c, o.blob);
        const bool runs = std::any_of(sw.segs.begin(), sw.segs.end(), [](const Sweep::Seg &g) { return g.wide_level < 0; });
        // algorithmic bytes of a launch solving `rows` rows with `nnz` stored entries:
        // values and column indices once, per row its pointer, level-list entry,
        // right-hand side and result (plus diagonal, fused addend and sum)
        const double vb = (double)sizeof(T);
        const double per_row = 8.0 + 2.0 * vb + (t.diag ? vb : 0.0) + (y2 ? 2.0 * vb : 0.0);
        auto bytes = [&](int64_t rows, int64_t nnz) { return (4.0 + vb) * (double)nnz + per_row * (double)rows; };
        if (runs) {
            ProfScope pg(c, s, RSILU_PROF_K_GATHER, (double)c.n * (4.0 + 2.0 * vb) * (y2 ? 2.0 : 1.0));
            launch_gather_lo<T>(s, (int32_t)c.n, t.rows, rhs, W.lo_rhs, add, y2 ? W.lo_add : nullptr, done);
        }
        for (const Sweep::Seg &g : sw.segs) {
            if (g.wide_level >= 0) {
                ProfScope pk(c, s, RSILU_PROF_K_LEVEL, bytes(g.rows, g.nnz));
                launch_trsv_level<T>(s, t, lv.ptr[g.wide_level], lv.ptr[(size_t)g.wide_level + 1], rhs, x, add, y2,
                                     done);
            } else {
                const int64_t off = sw.batch_off[(size_t)g.b0];
                const int32_t size = (int32_t)(sw.batch_off[(size_t)g.b0 + 1] - off);
                const int32_t *h0 = reinterpret_cast<const int32_t *>(sw.blob.data() + off);
                ProfScope pk(c, s, RSILU_PROF_K_SWEEP, bytes(g.rows, g.nnz));
                launch_trsv_sweep<T>(s, blob, off, size, h0[1], h0[6], g.b1 - g.b0, g.scheme, W.lo_rhs, x, W.lo_add, y2,
                                     done);
            }
        }
    } else if (c.prm.trsv == RSILU_TRSV_LEVELS) {
        for (int32_t l = 0; l < lv.nlev(); ++l)
            launch_trsv_level<T>(s, t, lv.ptr[l], lv.ptr[(size_t)l + 1], rhs, x, add, y2, done);
    } else {
        if constexpr (std::is_same<T, double>::value) launch_trsv_syncfree(s, t, rhs, x, add, y2, P.st, ticket, done);
    }
}

// Product with the explicit Y~ (yt = false: y = epi(Y~ x), rows m - n) or with
// Y~^T (yt = true: rows n), timed as one launch of its kernel class.
template <class T>
void spmv_y(Ctx &c, hipStream_t s, const Ptrs &P, const Pre<T> &W, bool yt, const T *x, T *y, const T *aux,
            Epi epi, const int32_t *done)
{
    const DCsrT<T> &a = yt ? W.YT : W.Y;
    const DevCsrOff &o = yt ? c.lay.YT : c.lay.Y;
    // values and column indices once, the row pointers, the gathered input and the output (plus aux)
    const double vb = (double)sizeof(T);
    const double bytes = (4.0 + vb) * (double)o.nnz + 4.0 * (o.nrows + 1) + vb * (double)o.ncols +
                         vb * (double)o.nrows * (aux ? 2.0 : 1.0);
    ProfScope pk(c, s, RSILU_PROF_K_SPMV_Y, bytes);
    launch_spmv<T>(s, a, yt ? P.pYT : P.pY, x, y, aux, epi, FIN_NONE, P.partials, W.segpart, P.st, done);
}

// Step 2 of Algorithm 3 / step 3 of Algorithm 2 with S^ by CG: u <- w after
// cg_steps steps of unpreconditioned CG on S~ w = u from w = 0, with
// S~ d = d + L2 (L1^{-1} (L1^{-T} (L2^T d))), or d + Y~ (Y~^T d) with the explicit
// Y~ (Section 3.2). The scalars stay on
// the device; a zero residual makes the remaining steps leave w unchanged.
// Temporaries: g, c2 and s2 (free at this point in both forms).
void cg_solve_S(Ctx &c, hipStream_t s, const Ptrs &P, const Pre<double> &W, const int32_t *done)
{
    const int32_t n = (int32_t)c.n, k = c.L2.nrows;
    double *w = at<double>(c, c.lay.cg_w), *res = at<double>(c, c.lay.cg_r), *p = at<double>(c, c.lay.cg_p),
           *q = at<double>(c, c.lay.cg_q);
    ProfScope ps(c, s, RSILU_PROF_DENSE_S);
    // Jacobi preconditioning (RSILU_CG_JACOBI): z = D^{-1} res takes res's place in the inner
    // products and the directions; the scalar steps are the same
    const bool jac = c.lay.cg_d != 0;
    const double *dS = jac ? at<double>(c, c.lay.cg_d) : nullptr;
    double *z = jac ? at<double>(c, c.lay.cg_z) : res;
    // per-block partials: (p, q) of the current step, and (res, z) of two steps in turn
    // (step i writes rr[i & 1] and reads the previous step's rr[(i + 1) & 1])
    double *pq = at<double>(c, c.lay.cg_part);
    double *rr[2] = {pq + kCgParts, pq + 2 * kCgParts};
    if (jac)
        launch_pcg_init(s, k, W.u, dS, w, res, z, p, done);
    else
        launch_cg_init(s, k, W.u, w, res, p, done);
    launch_cg_dot(s, k, res, z, rr[1], done);
    for (int32_t i = 0; i < c.prm.cg_steps; ++i) {
        if (yexplicit(c)) {
            // q = p + Y~ (Y~^T p)
            spmv_y<double>(c, s, P, W, true, p, W.g, nullptr, EPI_PLAIN, done);
            spmv_y<double>(c, s, P, W, false, W.g, q, p, EPI_ADD, done);
        } else {
            launch_spmv<double>(s, W.L2T, P.pL2T, p, W.g, nullptr, EPI_PLAIN, FIN_NONE, P.partials, W.segpart, P.st,
                                done);
            trsv<double>(c, s, P, W, W.L1b, c.lvL1T, c.swL1T, c.lay.L1b, W.g, W.c2, nullptr, nullptr, 1, done,
                         RSILU_PROF_TRSV_L1T);
            trsv<double>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, W.c2, W.s2, nullptr, nullptr, 2, done,
                         RSILU_PROF_TRSV_L1);
            launch_spmv<double>(s, W.L2, P.pL2, W.s2, q, p, EPI_ADD, FIN_NONE, P.partials, W.segpart, P.st, done);
        }
        launch_cg_dot(s, k, p, q, pq, done);
        double *rr_old = rr[(i + 1) & 1], *rr_new = rr[i & 1];
        if (i + 1 < c.prm.cg_steps) {
            // alpha, the update with the partials of res . z; then beta and p = z + beta p
            if (jac)
                launch_pcg_update_dot(s, k, p, q, dS, w, res, z, pq, rr_old, rr_new, done);
            else
                launch_cg_update_dot(s, k, p, q, w, res, pq, rr_old, rr_new, done);
            launch_cg_dir(s, k, z, p, rr_old, rr_new, done);
        } else {
            launch_cg_update(s, k, p, q, w, res, pq, rr_old, done);
        }
    }
    launch_copy(s, k, w, W.u, done);
    (void)n;
}

// Step 2 of Algorithm 3 / step 3 of Algorithm 2 with S^ by Chebyshev (RSILU_S_CHEB):
// u <- w after cheb_K steps of the Chebyshev iteration on S~ w = u over [1, cheb_b]
// from w = 0, each step one product with S~ (two with the explicit Y~; L2^T, two
// sweeps and L2 otherwise) and one fused vector update; the coefficients are fixed
// at setup, so no scalar is computed on the device. Temporaries: g, c2, s2 and the
// four (m - n)-vectors of the CG steps.
template <class T>
void cheb_solve_S(Ctx &c, hipStream_t s, const Ptrs &P, const Pre<T> &W, const int32_t *done)
{
    const int32_t k = c.L2.nrows;
    if (c.cheb_K == 0 || k == 0) return;  // S~ = I: w = u
    T *w = at<T>(c, c.lay.cg_w), *r = at<T>(c, c.lay.cg_r), *d = at<T>(c, c.lay.cg_p), *q = at<T>(c, c.lay.cg_q);
    ProfScope ps(c, s, RSILU_PROF_DENSE_S);
    launch_cheb_init<T>(s, k, W.u, r, d, w, c.cheb_theta, c.cheb_omega, done);
    for (int32_t j = 0; j < c.cheb_K; ++j) {
        if (yexplicit(c)) {
            spmv_y<T>(c, s, P, W, true, d, W.g, nullptr, EPI_PLAIN, done);
            spmv_y<T>(c, s, P, W, false, W.g, q, nullptr, EPI_PLAIN, done);
        } else {
            launch_spmv<T>(s, W.L2T, P.pL2T, d, W.g, nullptr, EPI_PLAIN, FIN_NONE, P.partials, W.segpart, P.st, done);
            trsv<T>(c, s, P, W, W.L1b, c.lvL1T, c.swL1T, c.lay.L1b, W.g, W.c2, nullptr, nullptr, 1, done,
                    RSILU_PROF_TRSV_L1T);
            trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, W.c2, W.s2, nullptr, nullptr, 2, done,
                    RSILU_PROF_TRSV_L1);
            launch_spmv<T>(s, W.L2, P.pL2, W.s2, q, nullptr, EPI_PLAIN, FIN_NONE, P.partials, W.segpart, P.st, done);
        }
        launch_cheb_update<T>(s, k, q, r, d, w, j + 1 == c.cheb_K ? W.u : nullptr, c.cheb_c1[(size_t)j],
                              c.cheb_c2[(size_t)j], done);
    }
}

// Algorithm 3 on the residual r (pivot order) -> hout, in precision T. For
// sync-free solves the outputs t, gp, v and hout must have been
// sentinel-filled, tickets cleared.
template <class T>
void apply_alg3(Ctx &c, hipStream_t s, const Ptrs &P, const Pre<T> &W, const T *r, T *hout, const int32_t *done)
{
    const int32_t n = (int32_t)c.n, k = c.L2.nrows;
    if (yexplicit(c) && k > 0 && c.smode != RSILU_S_NONE) {
        // explicit Y~: u = r2 - Y~ r1, S^ w = u, y = r1 + Y~^T w, L1 v = y, U h = v; u and w
        // in the device order of Y~'s rows (r2 gathered into it first)
        T *r2 = at<T>(c, c.lay.yk);
        launch_gather_lo<T>(s, k, at<int32_t>(c, c.lay.yperm), r + n, r2, nullptr, nullptr, done);
        spmv_y<T>(c, s, P, W, false, r, W.u, r2, EPI_SUB, done);
        if constexpr (std::is_same<T, double>::value) {
            if (c.smode == RSILU_S_CG) cg_solve_S(c, s, P, W, done);
        }
        if (c.smode == RSILU_S_CHEB) cheb_solve_S<T>(c, s, P, W, done);
        spmv_y<T>(c, s, P, W, true, W.u, W.y, r, EPI_ADD, done);
        trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, W.y, W.v, nullptr, nullptr, 2, done, RSILU_PROF_TRSV_L1);
        trsv<T>(c, s, P, W, W.Ub, c.lvU, c.swU, c.lay.Ub, W.v, hout, nullptr, nullptr, 3, done, RSILU_PROF_TRSV_U);
        return;
    }
    // step 1: u = r2 - Y r1 with Y r1 = L2 (L1^{-1} r1)
    trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, r, W.t, nullptr, nullptr, 0, done, RSILU_PROF_TRSV_L1);
    if (k == 0 || c.smode == RSILU_S_NONE) {
        // no A2 or no correction (w = 0): h = U^{-1} L1^{-1} r1
        trsv<T>(c, s, P, W, W.Ub, c.lvU, c.swU, c.lay.Ub, W.t, hout, nullptr, nullptr, 3, done, RSILU_PROF_TRSV_U);
        return;
    }
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_L2);
        launch_spmv<T>(s, W.L2, P.pL2, W.t, W.u, r + n, EPI_SUB, FIN_NONE, P.partials, W.segpart, P.st, done);
    }
    // step 2: S^ w = u (in place in u)
    if constexpr (std::is_same<T, double>::value) {
        if (c.smode == RSILU_S_DENSE) {
            ProfScope ps(c, s, RSILU_PROF_DENSE_S);
            launch_dense_chol_solve(s, k, P.sfac, W.u, done);
        } else if (c.smode == RSILU_S_CG) {
            cg_solve_S(c, s, P, W, done);
        }
    }
    if (c.smode == RSILU_S_CHEB) cheb_solve_S<T>(c, s, P, W, done);
    // step 3: y = r1 + Y^T w with Y^T w = L1^{-T} (L2^T w)
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_L2T);
        launch_spmv<T>(s, W.L2T, P.pL2T, W.u, W.g, nullptr, EPI_PLAIN, FIN_NONE, P.partials, W.segpart, P.st, done);
    }
    trsv<T>(c, s, P, W, W.L1b, c.lvL1T, c.swL1T, c.lay.L1b, W.g, W.gp, r, W.y, 1, done, RSILU_PROF_TRSV_L1T);
    // step 4: L1 v = y, U h = v
    trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, W.y, W.v, nullptr, nullptr, 2, done, RSILU_PROF_TRSV_L1);
    trsv<T>(c, s, P, W, W.Ub, c.lvU, c.swU, c.lay.Ub, W.v, hout, nullptr, nullptr, 3, done, RSILU_PROF_TRSV_U);
}

// Whether Algorithm 2 carries the M_b correction (six triangular sweeps
// instead of four).
bool alg2_correction(const Ctx &c) { return c.L2.nrows > 0 && c.smode != RSILU_S_NONE; }

// Sync-free outputs to sentinel-fill before one preconditioner application.
void fill_targets(const Ctx &c, const Ptrs &P, double *hout, double *f[4])
{
    f[0] = P.t;
    f[1] = P.gp;
    f[2] = P.v;
    f[3] = (c.prm.form == RSILU_FORM_ALG2 && alg2_correction(c)) ? P.c2 : hout;
}

// Algorithm 2 with k = n on z (pivot-order coordinates) -> hout, with
// M_a = (L1 U)^T (L1 U) for C1 and A2 represented by L2 U:
//   step 1  u_a = M_a^{-1} z, kept factored: g = L1^{-T} U^{-T} z, u_a = U^{-1} L1^{-1} g
//   step 2  w_b = A2 u_a = L2 L1^{-1} g
//   step 3  M_b v_b = w_b   (S~ dense, S^ = I, or skipped: v_b = 0)
//   step 4  w_a = z - A2^T v_b = z - U^T L2^T v_b
//   step 5  h = M_a^{-1} w_a = U^{-1} L1^{-1} (g - L1^{-T} L2^T v_b)
// so U^{-T} of step 5 cancels the U^T of step 4 and g is shared.
template <class T>
void apply_alg2(Ctx &c, hipStream_t s, const Ptrs &P, const Pre<T> &W, const T *z, T *hout, const int32_t *done)
{
    const int32_t n = (int32_t)c.n, k = c.L2.nrows;
    trsv<T>(c, s, P, W, W.UTf, c.lvUT, c.swUT, c.lay.UTf, z, W.t, nullptr, nullptr, 0, done, RSILU_PROF_TRSV_UT);
    trsv<T>(c, s, P, W, W.L1b, c.lvL1T, c.swL1T, c.lay.L1b, W.t, W.gp, nullptr, nullptr, 1, done, RSILU_PROF_TRSV_L1T);
    if (!alg2_correction(c)) {
        trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, W.gp, W.v, nullptr, nullptr, 2, done, RSILU_PROF_TRSV_L1);
        trsv<T>(c, s, P, W, W.Ub, c.lvU, c.swU, c.lay.Ub, W.v, hout, nullptr, nullptr, 3, done, RSILU_PROF_TRSV_U);
        return;
    }
    if (yexplicit(c)) {
        // explicit Y~ (A2 M_a^{-1} = Y~ L1^{-T} U^{-T}): w_b = Y~ g, v_b = M_b^{-1} w_b,
        // h = U^{-1} L1^{-1} (g - Y~^T v_b)
        spmv_y<T>(c, s, P, W, false, W.gp, W.u, nullptr, EPI_PLAIN, done);
        if constexpr (std::is_same<T, double>::value) {
            if (c.smode == RSILU_S_CG) cg_solve_S(c, s, P, W, done);
        }
        if (c.smode == RSILU_S_CHEB) cheb_solve_S<T>(c, s, P, W, done);
        spmv_y<T>(c, s, P, W, true, W.u, W.y, W.gp, EPI_SUB, done);
        trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, W.y, W.s2, nullptr, nullptr, 0, done, RSILU_PROF_TRSV_L1);
        trsv<T>(c, s, P, W, W.Ub, c.lvU, c.swU, c.lay.Ub, W.s2, hout, nullptr, nullptr, 1, done, RSILU_PROF_TRSV_U);
        return;
    }
    // step 2: w_b = L2 (L1^{-1} g) into u
    trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, W.gp, W.v, nullptr, nullptr, 2, done, RSILU_PROF_TRSV_L1);
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_L2);
        launch_spmv<T>(s, W.L2, P.pL2, W.v, W.u, nullptr, EPI_PLAIN, FIN_NONE, P.partials, W.segpart, P.st, done);
    }
    // step 3: v_b = M_b^{-1} w_b in place
    if constexpr (std::is_same<T, double>::value) {
        if (c.smode == RSILU_S_DENSE) {
            ProfScope ps(c, s, RSILU_PROF_DENSE_S);
            launch_dense_chol_solve(s, k, P.sfac, W.u, done);
        } else if (c.smode == RSILU_S_CG) {
            cg_solve_S(c, s, P, W, done);
        }
    }
    if (c.smode == RSILU_S_CHEB) cheb_solve_S<T>(c, s, P, W, done);
    // steps 4-5: y = g + L1^{-T} (-L2^T v_b), then L1 s2 = y, U h = s2
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_L2T);
        launch_spmv<T>(s, W.L2T, P.pL2T, W.u, W.g, nullptr, EPI_NEG, FIN_NONE, P.partials, W.segpart, P.st, done);
    }
    trsv<T>(c, s, P, W, W.L1b, c.lvL1T, c.swL1T, c.lay.L1b, W.g, W.c2, W.gp, W.y, 3, done, RSILU_PROF_TRSV_L1T);
    if constexpr (std::is_same<T, double>::value) {
        if (syncfree(c)) launch_refill(s, n, W.s2, hout, P.st, done);
    }
    trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, W.y, W.s2, nullptr, nullptr, 0, done, RSILU_PROF_TRSV_L1);
    trsv<T>(c, s, P, W, W.Ub, c.lvU, c.swU, c.lay.Ub, W.s2, hout, nullptr, nullptr, 1, done, RSILU_PROF_TRSV_U);
}

// h = M^{-1} z of one iteration, in the configured form and precision. The
// FP32 preconditioner converts its input (r or z) to FP32 and h back to FP64.
void apply_form(Ctx &c, hipStream_t s, const Ptrs &P, double *hout, const int32_t *done)
{
    const bool a2 = c.prm.form == RSILU_FORM_ALG2;
    if (fp32(c)) {
        const Pre<float> W = pre<float>(c);
        float *in = at<float>(c, c.lay.f32a), *out = at<float>(c, c.lay.f32b);
        if (a2) {
            launch_cvt(s, (int32_t)c.n, P.z, in, done);
            apply_alg2<float>(c, s, P, W, in, out, done);
        } else {
            launch_cvt(s, (int32_t)c.m, P.r, in, done);
            apply_alg3<float>(c, s, P, W, in, out, done);
        }
        launch_cvt(s, (int32_t)c.n, out, hout, done);
        return;
    }
    const Pre<double> W = pre<double>(c);
    if (a2) {
        apply_alg2<double>(c, s, P, W, P.z, hout, done);
        if (c.R.nrows > 0) {
            // removed rows (Section 3.4): h = g + M^{-1} R^T W^{-1} R g with g = M^{-1} z
            const Layout &L = c.lay;
            double *wr = at<double>(c, L.wr), *wz = at<double>(c, L.wz), *wh = at<double>(c, L.wh);
            launch_spmv<double>(s, dcsr(c, L.R), dplan(c, L.pR), hout, wr, nullptr, EPI_PLAIN, FIN_NONE, P.partials,
                                P.segpart, P.st, done);
            launch_dense_chol_solve(s, c.R.nrows, at<double>(c, L.wfac), wr, done);
            launch_spmv<double>(s, dcsr(c, L.RT), dplan(c, L.pRT), wr, wz, nullptr, EPI_PLAIN, FIN_NONE, P.partials,
                                P.segpart, P.st, done);
            apply_alg2<double>(c, s, P, W, wz, wh, done);
            launch_add(s, (int32_t)c.n, wh, hout, done);
        }
    } else {
        apply_alg3<double>(c, s, P, W, P.r, hout, done);
    }
}

template <class T>
void trsv_which(Ctx &c, hipStream_t s, const Ptrs &P, const Pre<T> &W, int32_t which, const T *rhs, T *x)
{
    switch (which) {
    case 0: trsv<T>(c, s, P, W, W.L1f, c.lvL1, c.swL1, c.lay.L1f, rhs, x, nullptr, nullptr, 0, nullptr, RSILU_PROF_TRSV_L1); break;
    case 1: trsv<T>(c, s, P, W, W.L1b, c.lvL1T, c.swL1T, c.lay.L1b, rhs, x, nullptr, nullptr, 0, nullptr, RSILU_PROF_TRSV_L1T); break;
    case 2: trsv<T>(c, s, P, W, W.Ub, c.lvU, c.swU, c.lay.Ub, rhs, x, nullptr, nullptr, 0, nullptr, RSILU_PROF_TRSV_U); break;
    default: trsv<T>(c, s, P, W, W.UTf, c.lvUT, c.swUT, c.lay.UTf, rhs, x, nullptr, nullptr, 0, nullptr, RSILU_PROF_TRSV_UT); break;
    }
}

// LSQR in the M-inner-product form (rsilu.h, RSILU_KRYLOV_LSQR). Vectors: u in r,
// t in q (m); s in z (the Algorithm 2 input), h in h, x_hat in xh; v, M v and w
// in their own n-vectors.
void enqueue_lsqr_init(Ctx &c, hipStream_t s, const Ptrs &P, const double *b)
{
    const int32_t n = (int32_t)c.n, m = (int32_t)c.m;
    double *v = at<double>(c, c.lay.l_v), *Mv = at<double>(c, c.lay.l_mv), *w = at<double>(c, c.lay.l_w);
    launch_gather(s, m, n, P.perm, b, P.r, P.xh, nullptr);
    launch_dot(s, m, P.r, P.r, FIN_L_BETA1, P.partials, P.st, P.done);
    launch_lsqr_scale(s, m, P.r, P.r, P.st, P.done);
    launch_spmv<double>(s, P.AT, P.pAT, P.r, P.z, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, P.done);
    launch_lsqr_s(s, n, P.z, nullptr, P.colnorm, FIN_L_S1, P.partials, P.st, P.done);
    apply_form(c, s, P, P.h, P.done);
    launch_dot(s, n, P.z, P.h, FIN_L_ALPHA0, P.partials, P.st, P.done);
    launch_lsqr_v(s, n, P.h, P.z, P.xh, v, Mv, w, true, P.st, P.done);
}

void enqueue_lsqr_iteration(Ctx &c, hipStream_t s, const Ptrs &P)
{
    const int32_t n = (int32_t)c.n, m = (int32_t)c.m;
    double *v = at<double>(c, c.lay.l_v), *Mv = at<double>(c, c.lay.l_mv), *w = at<double>(c, c.lay.l_w);
    // t = A_hat v - alpha u, beta = ||t||, u = t / beta
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_A);
        launch_spmv<double>(s, P.A, P.pA, v, P.q, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, P.done);
    }
    launch_lsqr_t(s, m, P.r, P.q, FIN_L_BETA, P.partials, P.st, P.done);
    launch_lsqr_scale(s, m, P.q, P.r, P.st, P.done);
    // s = A_hat^T u - beta M v with ||D^{-1} s||
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_AT);
        launch_spmv<double>(s, P.AT, P.pAT, P.r, P.z, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st,
                            P.done);
    }
    launch_lsqr_s(s, n, P.z, Mv, P.colnorm, FIN_L_SNORM, P.partials, P.st, P.done);
    // h = M^{-1} s, alpha = sqrt(s . h), the Givens step and the stop test
    apply_form(c, s, P, P.h, P.done);
    launch_dot(s, n, P.z, P.h, FIN_L_ALPHA, P.partials, P.st, P.done);
    // x_hat, v, M v, w; then a requested stop takes effect
    launch_lsqr_v(s, n, P.h, P.z, P.xh, v, Mv, w, false, P.st, P.done);
    launch_lsqr_commit(s, P.st);
}

void enqueue_iteration(Ctx &c, hipStream_t s, const Ptrs &P)
{
    const int32_t n = (int32_t)c.n, m = (int32_t)c.m;
    // q = A p, alpha = rho / (q, q)
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_A);
        launch_spmv<double>(s, P.A, P.pA, P.p, P.q, nullptr, EPI_SQ, FIN_ALPHA, P.partials, P.segpart, P.st, P.done);
    }
    // x += alpha p, r -= alpha q (and prepare the sync-free outputs)
    const bool sf = syncfree(c);
    double *f[4];
    fill_targets(c, P, P.h, f);
    launch_update(s, n, m, P.p, P.xh, P.q, P.r, sf ? f[0] : nullptr, f[1], f[2], f[3], P.st, P.done);
    // z = A^T r, stop test on ||D^{-1} z|| = ||A^T r||
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_AT);
        launch_spmv<double>(s, P.AT, P.pAT, P.r, P.z, P.colnorm, EPI_WSQ, FIN_STOP, P.partials, P.segpart, P.st, P.done);
    }
    // h = M^{-1} z by Algorithm 3 on (r1, r2) or Algorithm 2 on z
    apply_form(c, s, P, P.h, P.done);
    // rho' = (z, h), beta = rho'/rho, p = h + beta p
    launch_dot(s, n, P.z, P.h, FIN_BETA, P.partials, P.st, P.done);
    launch_pupdate(s, n, P.h, P.p, P.st, false, P.done);
}

// Capture `poll` iterations of the configured solver into a graph (on the
// handle's own stream, thread-local capture mode), for replay by rsilu_solve.
hipError_t capture_iterations(Ctx &c, const Ptrs &P)
{
    hipError_t e = hipSuccess;
    if (!c.cap_stream) {
        hipStream_t cs;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        c.cap_stream = cs;
    }
    hipStream_t cs = static_cast<hipStream_t>(c.cap_stream);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int i = 0; i < c.prm.poll; ++i) {
        if (c.prm.krylov == RSILU_KRYLOV_LSQR)
            enqueue_lsqr_iteration(c, cs, P);
        else
            enqueue_iteration(c, cs, P);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess) return e;
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    c.graph_exec = x;
    return hipSuccess;
}

}  // namespace

void release_graph(Ctx &c)
{
    if (c.graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(c.graph_exec));
    c.graph_exec = nullptr;
}

}  // namespace rsilu

using namespace rsilu;

extern "C" {

void rsilu_params_default(rsilu_params_t *p)
{
    if (!p) return;
    p->p = 10;
    p->tau = 1e-2;
    p->mu = 0.1;
    p->small = 1e-10;
    p->colscale = 1;
    p->smode = RSILU_S_AUTO;
    p->maxit = 2000;
    p->trsv = RSILU_TRSV_HYBRID;
    p->poll = 8;
    p->form = RSILU_FORM_ALG3;
    p->precision = RSILU_PREC_FP64;
    p->cg_steps = 2;
    p->krylov = RSILU_KRYLOV_PCGLS;
    p->graph = 1;
    p->sweep = RSILU_SWEEP_AUTO;
    p->ystore = RSILU_Y_IMPLICIT;
    p->ytau = 1e-2;
    p->poly_degree = 0;
    p->poly_delta = 0.9;
    p->cg_precond = RSILU_CG_NONE;
    p->reserved3 = 0;
}

const char *rsilu_status_string(rsilu_status_t s)
{
    switch (s) {
    case RSILU_OK: return "ok";
    case RSILU_NOT_CONVERGED: return "not converged within maxit iterations";
    case RSILU_BREAKDOWN: return "breakdown (zero or non-finite scalar)";
    case RSILU_EINVAL: return "invalid argument";
    case RSILU_ENOMEM: return "out of memory or device buffer too small";
    case RSILU_EHIP: return "HIP runtime error";
    case RSILU_ESTATE: return "call out of order";
    case RSILU_EINTERNAL: return "internal wait bound exceeded in a kernel";
    }
    return "unknown status";
}

rsilu_status_t rsilu_factor(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
                            const rsilu_params_t *params, rsilu_handle_t *out)
{
    if (!out) return RSILU_EINVAL;
    *out = nullptr;
    rsilu_ctx *c = nullptr;
    try {
        c = new rsilu_ctx();
        if (params)
            c->prm = *params;
        else
            rsilu_params_default(&c->prm);
        rsilu_status_t st = build_factorization(*c, m, n, rowptr, colind, val);
        if (st != RSILU_OK) {
            delete c;
            return st;
        }
        plan_layout(*c);
    } catch (const std::bad_alloc &) {
        delete c;
        return RSILU_ENOMEM;
    } catch (...) {
        delete c;
        return RSILU_EINVAL;
    }
    *out = c;
    return RSILU_OK;
}

size_t rsilu_device_bytes(rsilu_handle_t h) { return h ? h->lay.total : 0; }

rsilu_status_t rsilu_get_stats(rsilu_handle_t h, rsilu_stats_t *s)
{
    if (!h || !s) return RSILU_EINVAL;
    std::memset(s, 0, sizeof(*s));
    s->m = h->m;
    s->n = h->n;
    s->nnz_a = h->nnz_a;
    s->nnz_l1 = h->L1.nnz();
    s->nnz_l2 = h->L2.nnz();
    s->nnz_u = h->U.nnz();
    const int64_t k = h->L2.nrows;
    s->psize = s->nnz_l1 + s->nnz_l2 + s->nnz_u + h->n + (h->smode == RSILU_S_DENSE ? k * (k + 1) / 2 : 0);
    s->nmod = h->nmod;
    s->levels_l1 = h->lvL1.nlev();
    s->levels_l1t = h->lvL1T.nlev();
    s->levels_u = h->lvU.nlev();
    s->levels_ut = h->lvUT.nlev();
    s->smode = h->smode;
    s->sweep_schemes = 0;
    const Sweep *sws[4] = {&h->swL1, &h->swL1T, &h->swU, &h->swUT};
    for (int f = 0; f < 4; ++f)
        for (const Sweep::Seg &g : sws[f]->segs)
            s->sweep_schemes |= (g.wide_level >= 0 ? 0x80 : (1 << (g.scheme & 7))) << (8 * f);
    s->device_bytes = h->lay.total;
    s->nnz_y = yexplicit(*h) ? h->Y.nnz() : 0;
    s->cheb_b = h->cheb_b;
    s->cheb_degree = h->cheb_K;
    s->cheb_scale = h->cheb_omega;
    return RSILU_OK;
}

rsilu_status_t rsilu_get_perm(rsilu_handle_t h, int32_t *perm)
{
    if (!h || !perm) return RSILU_EINVAL;
    std::copy(h->perm.begin(), h->perm.end(), perm);
    return RSILU_OK;
}

rsilu_status_t rsilu_get_colnorm(rsilu_handle_t h, double *cn)
{
    if (!h || !cn) return RSILU_EINVAL;
    std::copy(h->colnorm.begin(), h->colnorm.end(), cn);
    return RSILU_OK;
}

static const Csr *factor_of(rsilu_handle_t h, int32_t which)
{
    switch (which) {
    case 0: return &h->L1;
    case 1: return &h->L2;
    case 2: return &h->U;
    case 3: return &h->Ahat;
    case 5: return yexplicit(*h) ? &h->Y : nullptr;
    default: return nullptr;
    }
}

int64_t rsilu_factor_nnz(rsilu_handle_t h, int32_t which)
{
    if (!h) return -1;
    if (which == 4) return h->n;
    const Csr *a = factor_of(h, which);
    return a ? a->nnz() : -1;
}

rsilu_status_t rsilu_get_factor(rsilu_handle_t h, int32_t which, int64_t *rowptr, int32_t *col, double *val)
{
    if (!h || !val) return RSILU_EINVAL;
    if (which == 4) {
        std::copy(h->Udiag.begin(), h->Udiag.end(), val);
        return RSILU_OK;
    }
    const Csr *a = factor_of(h, which);
    if (!a || !rowptr || !col) return RSILU_EINVAL;
    for (size_t i = 0; i < a->ptr.size(); ++i) rowptr[i] = a->ptr[i];
    std::copy(a->col.begin(), a->col.end(), col);
    std::copy(a->val.begin(), a->val.end(), val);
    return RSILU_OK;
}

rsilu_status_t rsilu_get_levels(rsilu_handle_t h, int32_t which, int32_t *level_ptr, int32_t *level_rows)
{
    if (!h || !level_ptr || !level_rows) return RSILU_EINVAL;
    const Levels *lv = nullptr;
    switch (which) {
    case 0: lv = &h->lvL1; break;
    case 1: lv = &h->lvL1T; break;
    case 2: lv = &h->lvU; break;
    case 3: lv = &h->lvUT; break;
    default: return RSILU_EINVAL;
    }
    std::copy(lv->ptr.begin(), lv->ptr.end(), level_ptr);
    std::copy(lv->rows.begin(), lv->rows.end(), level_rows);
    return RSILU_OK;
}

rsilu_status_t rsilu_upload(rsilu_handle_t h, void *dev_buf, size_t bytes, hipStream_t s)
{
    if (!h || !dev_buf) return RSILU_EINVAL;
    release_graph(*h);  // a captured graph holds the previous buffer's addresses
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255u) != 0) return RSILU_EINVAL;
    if (bytes < h->lay.total) return RSILU_ENOMEM;
    Ctx &c = *h;
    c.dev = dev_buf;
    c.dev_bytes = bytes;
    RSILU_HIP(hipGetDevice(&c.device));
    if (!c.pinned) RSILU_HIP(hipHostMalloc(&c.pinned, sizeof(PinnedMail), hipHostMallocDefault));
    const Layout &L = c.lay;
    auto put = [&](size_t off, const void *src, size_t nbytes) -> hipError_t {
        if (nbytes == 0) return hipSuccess;
        return hipMemcpyAsync(static_cast<char *>(c.dev) + off, src, nbytes, hipMemcpyHostToDevice, s);
    };
    // FP32 copies of factor values live until the copies are done (synchronised below)
    std::vector<std::vector<float>> f32hold;
    auto put_vals = [&](size_t off, const std::vector<double> &v, int32_t vbytes) -> hipError_t {
        if (vbytes == 8) return put(off, v.data(), v.size() * sizeof(double));
        f32hold.emplace_back(v.begin(), v.end());
        return put(off, f32hold.back().data(), v.size() * sizeof(float));
    };
    auto put_csr = [&](const DevCsrOff &o, const Csr &a) -> hipError_t {
        hipError_t e = put(o.ptr, a.ptr.data(), a.ptr.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.col, a.col.data(), a.col.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put_vals(o.val, a.val, o.vbytes);
        return e;
    };
    auto put_plan = [&](const DevPlanOff &o, const SpmvPlan &p) -> hipError_t {
        hipError_t e = put(o.long_rows, p.long_rows.data(), p.long_rows.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.seg_ptr, p.seg_ptr.data(), p.seg_ptr.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.seg_beg, p.seg_beg.data(), p.seg_beg.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.seg_end, p.seg_end.data(), p.seg_end.size() * sizeof(int32_t));
        return e;
    };
    auto put_tri = [&](const DevTriOff &o, const Csr &a, const std::vector<double> *diag, const Levels &lv,
                       const Chunks &ch, const LoTri &lo) -> hipError_t {
        hipError_t e = put_csr(o.a, a);
        if (e == hipSuccess && diag) e = put_vals(o.diag, *diag, o.a.vbytes);
        if (e == hipSuccess) e = put(o.rows, lv.rows.data(), lv.rows.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.chunk, ch.ptr.data(), ch.ptr.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.lev, lv.ptr.data(), lv.ptr.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put_csr(o.lo, lo.a);
        if (e == hipSuccess && o.ldiag) e = put_vals(o.ldiag, lo.diag, o.lo.vbytes);
        if (e == hipSuccess) e = put(o.lrec, lo.rec.data(), lo.rec.size());
        return e;
    };
    auto put_sweep = [&](const DevTriOff &o, const Sweep &sw) -> hipError_t {
        return put(o.blob, sw.blob.data(), sw.blob.size());
    };
    RSILU_HIP(put_csr(L.A, c.Ahat));
    RSILU_HIP(put_csr(L.AT, c.AhatT));
    RSILU_HIP(put_csr(L.L2, c.L2));
    RSILU_HIP(put_csr(L.L2T, c.L2T));
    RSILU_HIP(put_plan(L.pA, c.plA));
    RSILU_HIP(put_plan(L.pAT, c.plAT));
    RSILU_HIP(put_plan(L.pL2, c.plL2));
    RSILU_HIP(put_plan(L.pL2T, c.plL2T));
    if (yexplicit(c)) {
        RSILU_HIP(put_csr(L.Y, c.Yd));
        RSILU_HIP(put_csr(L.YT, c.YdT));
        RSILU_HIP(put(L.yperm, c.yperm.data(), c.yperm.size() * sizeof(int32_t)));
        RSILU_HIP(put(L.yperm_inv, c.yperm_inv.data(), c.yperm_inv.size() * sizeof(int32_t)));
        RSILU_HIP(put_plan(L.pY, c.plY));
        RSILU_HIP(put_plan(L.pYT, c.plYT));
    }
    RSILU_HIP(put_tri(L.L1f, c.L1, nullptr, c.lvL1, c.chL1, c.loL1));
    RSILU_HIP(put_tri(L.L1b, c.L1T, nullptr, c.lvL1T, c.chL1T, c.loL1T));
    RSILU_HIP(put_tri(L.Ub, c.U, &c.Udiag, c.lvU, c.chU, c.loU));
    RSILU_HIP(put_tri(L.UTf, c.UT, &c.Udiag, c.lvUT, c.chUT, c.loUT));
    RSILU_HIP(put_sweep(L.L1f, c.swL1));
    RSILU_HIP(put_sweep(L.L1b, c.swL1T));
    RSILU_HIP(put_sweep(L.Ub, c.swU));
    RSILU_HIP(put_sweep(L.UTf, c.swUT));
    RSILU_HIP(put(L.perm, c.perm.data(), c.perm.size() * sizeof(int32_t)));
    RSILU_HIP(put(L.colnorm, c.colnorm.data(), c.colnorm.size() * sizeof(double)));
    RSILU_HIP(put(L.sfac, c.sfac.data(), c.sfac.size() * sizeof(double)));
    if (L.cg_d) RSILU_HIP(put(L.cg_d, c.cg_diag.data(), c.cg_diag.size() * sizeof(double)));
    if (c.smode == RSILU_S_CHEB) {
        RSILU_HIP(put(L.cheb, c.cheb_c1.data(), c.cheb_c1.size() * sizeof(double)));
        RSILU_HIP(put(L.cheb + sizeof(double) * c.cheb_c1.size(), c.cheb_c2.data(), c.cheb_c2.size() * sizeof(double)));
    }
    if (c.R.nrows > 0) {
        RSILU_HIP(put_csr(L.R, c.R));
        RSILU_HIP(put_csr(L.RT, c.RT));
        RSILU_HIP(put_plan(L.pR, c.plR));
        RSILU_HIP(put_plan(L.pRT, c.plRT));
        RSILU_HIP(put(L.wfac, c.wfac.data(), c.wfac.size() * sizeof(double)));
    }
    PinnedMail *mail = static_cast<PinnedMail *>(c.pinned);
    std::memset(&mail->init, 0, sizeof(DevState));
    RSILU_HIP(hipMemcpyAsync(at<DevState>(c, L.state), &mail->init, sizeof(DevState), hipMemcpyHostToDevice, s));
    RSILU_HIP(hipStreamSynchronize(s));
    return RSILU_OK;
}

rsilu_status_t rsilu_add_rows(rsilu_handle_t h, int64_t count, const int64_t *rowptr, const int32_t *colind,
                              const double *val)
{
    if (!h) return RSILU_EINVAL;
    Ctx &c = *h;
    try {
        const rsilu_status_t rc = append_rows(c, count, rowptr, colind, val);
        if (rc != RSILU_OK) return rc;
        plan_layout(c);
    } catch (const std::bad_alloc &) {
        return RSILU_ENOMEM;
    }
    release_graph(c);  // the captured iterations hold the old layout's addresses
    c.dev = nullptr;   // the layout grew: upload again before the next solve
    c.dev_bytes = 0;
    return RSILU_OK;
}

rsilu_status_t rsilu_remove_rows(rsilu_handle_t h, int64_t count, const int64_t *rows)
{
    if (!h) return RSILU_EINVAL;
    Ctx &c = *h;
    try {
        const rsilu_status_t rc = remove_rows(c, count, rows);
        if (rc != RSILU_OK) return rc;
        plan_layout(c);
    } catch (const std::bad_alloc &) {
        return RSILU_ENOMEM;
    }
    release_graph(c);  // the captured iterations hold the old layout's addresses
    c.dev = nullptr;   // the layout changed: upload again before the next solve
    c.dev_bytes = 0;
    return RSILU_OK;
}

static rsilu_status_t check_ready(rsilu_handle_t h)
{
    if (!h) return RSILU_EINVAL;
    if (!h->dev) return RSILU_ESTATE;
    return RSILU_OK;
}

rsilu_status_t rsilu_solve(rsilu_handle_t h, const double *b, double tol, double *x, int32_t *iters,
                           double *atr_norm, double *atr_rel, hipStream_t s)
{
    rsilu_status_t rc = check_ready(h);
    if (rc != RSILU_OK) return rc;
    if (!b || !x || static_cast<const void *>(b) == static_cast<const void *>(x) || !(tol >= 0.0) ||
        !std::isfinite(tol))
        return RSILU_EINVAL;
    Ctx &c = *h;
    const Ptrs P = ptrs(c);
    const int32_t n = (int32_t)c.n, m = (int32_t)c.m;
    PinnedMail *mail = static_cast<PinnedMail *>(c.pinned);
    std::memset(&mail->init, 0, sizeof(DevState));
    mail->init.tol = tol;
    mail->init.maxit = c.prm.maxit;
    RSILU_HIP(hipMemcpyAsync(P.st, &mail->init, sizeof(DevState), hipMemcpyHostToDevice, s));
    const bool sf = syncfree(c);
    const bool lsqr = c.prm.krylov == RSILU_KRYLOV_LSQR;

    // ---- initialisation: x0 = 0; PCGLS: r0 = P b, z0 = A^T r0, h0 = B(r0), rho0, p0 = h0
    // (LSQR: its own start, enqueue_lsqr_init)
    c.ev_iter = 0;
    c.ev_open.clear();
    c.ev_next = 0;
    if (lsqr) {
        enqueue_lsqr_init(c, s, P, b);
    } else {
        launch_gather(s, m, n, P.perm, b, P.r, P.xh, nullptr);
        launch_spmv<double>(s, P.AT, P.pAT, P.r, P.z, P.colnorm, EPI_WSQ, FIN_INIT, P.partials, P.segpart, P.st,
                            nullptr);
        if (sf) {
            double *f[4];
            fill_targets(c, P, P.h, f);
            launch_fill(s, n, f[0], f[1], f[2], f[3], P.st);
        }
        apply_form(c, s, P, P.h, P.done);
        launch_dot(s, n, P.z, P.h, FIN_RHO0, P.partials, P.st, P.done);
        launch_pupdate(s, n, P.h, P.p, P.st, true, P.done);
    }
    RSILU_HIP(hipGetLastError());

    // ---- iterations, polled every `poll` steps (maxit = 0 stops after the init). With
    // graphs, `poll` iterations are captured once per upload and replayed; iterations
    // past maxit or past convergence return at once on the device's stop flag.
    const bool use_graph = c.prm.graph && !c.prof;
    if (use_graph && !c.graph_exec) RSILU_HIP(capture_iterations(c, P));
    int64_t enqueued = 0;
    bool stop = c.prm.maxit == 0;
    while (!stop) {
        if (use_graph) {
            RSILU_HIP(hipGraphLaunch(static_cast<hipGraphExec_t>(c.graph_exec), s));
            enqueued += c.prm.poll;
        } else {
            const int batch = (int)std::min<int64_t>(c.prm.poll, (int64_t)c.prm.maxit - enqueued);
            for (int i = 0; i < batch; ++i) {
                c.ev_iter = (int)(enqueued + i + 1);
                if (lsqr)
                    enqueue_lsqr_iteration(c, s, P);
                else
                    enqueue_iteration(c, s, P);
            }
            enqueued += batch;
        }
        RSILU_HIP(hipGetLastError());
        RSILU_HIP(hipMemcpyAsync(&mail->poll, P.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        RSILU_HIP(hipStreamSynchronize(s));
        if (c.prof) prof_collect(c, mail->poll.done ? mail->poll.iter - 1 : mail->poll.iter);
        if (mail->poll.done || mail->poll.err || enqueued >= c.prm.maxit) stop = true;
    }

    // ---- exit: x = D x_hat; true ||A^T (b - A x)|| recomputed from x_hat
    launch_scale_out(s, n, P.xh, P.colnorm, x);
    launch_spmv<double>(s, P.A, P.pA, P.xh, P.q, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, nullptr);
    launch_residual(s, m, P.perm, b, P.q, P.r);
    launch_spmv<double>(s, P.AT, P.pAT, P.r, P.z, P.colnorm, EPI_WSQ, FIN_ATR, P.partials, P.segpart, P.st, nullptr);
    RSILU_HIP(hipGetLastError());
    RSILU_HIP(hipMemcpyAsync(&mail->poll, P.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    RSILU_HIP(hipStreamSynchronize(s));
    const DevState &st = mail->poll;
    if (iters) *iters = st.iter;
    if (atr_norm) *atr_norm = st.atr;
    if (atr_rel) *atr_rel = st.nb > 0.0 ? st.atr / st.nb : 0.0;
    if (st.err) return RSILU_EINTERNAL;
    if (st.status == 2) return RSILU_BREAKDOWN;
    if (c.prm.maxit == 0 && st.nb > 0.0) return RSILU_NOT_CONVERGED;
    if (st.status == 1 || (!st.done && st.nb > 0.0)) return RSILU_NOT_CONVERGED;
    return RSILU_OK;
}

rsilu_status_t rsilu_spmv(rsilu_handle_t h, int32_t op, const double *xin, double *y, hipStream_t s)
{
    rsilu_status_t rc = check_ready(h);
    if (rc != RSILU_OK) return rc;
    if (!xin || !y || static_cast<const void *>(xin) == static_cast<const void *>(y)) return RSILU_EINVAL;
    Ctx &c = *h;
    const Ptrs P = ptrs(c);
    const int32_t n = (int32_t)c.n, k = c.L2.nrows;
    switch (op) {
    case 0: launch_spmv<double>(s, P.A, P.pA, xin, y, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, nullptr); break;
    case 1: launch_spmv<double>(s, P.AT, P.pAT, xin, y, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, nullptr); break;
    case 2:
    case 3:
    case 4:
    case 5: {
        // products with L2, L2^T, Y~ and Y~^T in the preconditioner's precision
        if (op >= 4 && !yexplicit(c)) return RSILU_EINVAL;
        const bool fwd = op == 2 || op == 4;  // (m-n) x n operator
        const int32_t nin = fwd ? n : k, nout = fwd ? k : n;
        const DPlan &pl = op == 2 ? P.pL2 : op == 3 ? P.pL2T : op == 4 ? P.pY : P.pYT;
        // the device copy of Y~ holds its rows in yperm order: Y~ x is put back into the
        // user's row order, and Y~^T takes its input in the device order
        double *yk = op >= 4 ? at<double>(c, c.lay.yk) : nullptr;
        const int32_t *yp = op >= 4 ? at<int32_t>(c, c.lay.yperm) : nullptr;
        const int32_t *ypi = op >= 4 ? at<int32_t>(c, c.lay.yperm_inv) : nullptr;
        const double *src = xin;
        if (op == 5) {
            launch_gather_lo<double>(s, k, yp, xin, yk, nullptr, nullptr, nullptr);
            src = yk;
        }
        double *dst = op == 4 ? yk : y;
        if (fp32(c)) {
            const Pre<float> W = pre<float>(c);
            const DCsrT<float> &a = op == 2 ? W.L2 : op == 3 ? W.L2T : op == 4 ? W.Y : W.YT;
            float *in = at<float>(c, c.lay.f32a), *out = at<float>(c, c.lay.f32b);
            launch_cvt(s, nin, src, in, nullptr);
            launch_spmv<float>(s, a, pl, in, out, nullptr, EPI_PLAIN, FIN_NONE, P.partials, W.segpart, P.st, nullptr);
            launch_cvt(s, nout, out, dst, nullptr);
        } else {
            const Pre<double> W = pre<double>(c);
            const DCsrT<double> &a = op == 2 ? W.L2 : op == 3 ? W.L2T : op == 4 ? W.Y : W.YT;
            launch_spmv<double>(s, a, pl, src, dst, nullptr, EPI_PLAIN, FIN_NONE, P.partials, W.segpart, P.st, nullptr);
        }
        if (op == 4) launch_gather_lo<double>(s, k, ypi, yk, y, nullptr, nullptr, nullptr);
        break;
    }
    default: return RSILU_EINVAL;
    }
    RSILU_HIP(hipGetLastError());
    return RSILU_OK;
}

rsilu_status_t rsilu_trsv(rsilu_handle_t h, int32_t which, const double *rhs, double *x, hipStream_t s)
{
    rsilu_status_t rc = check_ready(h);
    if (rc != RSILU_OK) return rc;
    if (!rhs || !x || static_cast<const void *>(rhs) == static_cast<const void *>(x)) return RSILU_EINVAL;
    if (which < 0 || which > 3) return RSILU_EINVAL;
    Ctx &c = *h;
    const Ptrs P = ptrs(c);
    const int32_t n = (int32_t)c.n;
    if (fp32(c)) {
        float *in = at<float>(c, c.lay.f32a), *out = at<float>(c, c.lay.f32b);
        launch_cvt(s, n, rhs, in, nullptr);
        trsv_which<float>(c, s, P, pre<float>(c), which, in, out);
        launch_cvt(s, n, out, x, nullptr);
    } else {
        if (syncfree(c)) launch_fill(s, n, x, nullptr, nullptr, nullptr, P.st);
        trsv_which<double>(c, s, P, pre<double>(c), which, rhs, x);
    }
    RSILU_HIP(hipGetLastError());
    return RSILU_OK;
}

rsilu_status_t rsilu_apply(rsilu_handle_t h, const double *r, double *hout, hipStream_t s)
{
    rsilu_status_t rc = check_ready(h);
    if (rc != RSILU_OK) return rc;
    if (!r || !hout || static_cast<const void *>(r) == static_cast<const void *>(hout)) return RSILU_EINVAL;
    Ctx &c = *h;
    const Ptrs P = ptrs(c);
    if (fp32(c)) {
        float *in = at<float>(c, c.lay.f32a), *out = at<float>(c, c.lay.f32b);
        launch_cvt(s, (int32_t)c.m, r, in, nullptr);
        apply_alg3<float>(c, s, P, pre<float>(c), in, out, nullptr);
        launch_cvt(s, (int32_t)c.n, out, hout, nullptr);
    } else {
        if (syncfree(c)) launch_fill(s, (int32_t)c.n, P.t, P.gp, P.v, hout, P.st);
        apply_alg3<double>(c, s, P, pre<double>(c), r, hout, nullptr);
    }
    RSILU_HIP(hipGetLastError());
    return RSILU_OK;
}

rsilu_status_t rsilu_apply_z(rsilu_handle_t h, const double *z, double *hout, hipStream_t s)
{
    rsilu_status_t rc = check_ready(h);
    if (rc != RSILU_OK) return rc;
    if (!z || !hout || static_cast<const void *>(z) == static_cast<const void *>(hout)) return RSILU_EINVAL;
    Ctx &c = *h;
    const Ptrs P = ptrs(c);
    if (fp32(c)) {
        float *in = at<float>(c, c.lay.f32a), *out = at<float>(c, c.lay.f32b);
        launch_cvt(s, (int32_t)c.n, z, in, nullptr);
        apply_alg2<float>(c, s, P, pre<float>(c), in, out, nullptr);
        launch_cvt(s, (int32_t)c.n, out, hout, nullptr);
    } else {
        if (syncfree(c)) launch_fill(s, (int32_t)c.n, P.t, P.gp, P.v, alg2_correction(c) ? P.c2 : hout, P.st);
        apply_alg2<double>(c, s, P, pre<double>(c), z, hout, nullptr);
    }
    RSILU_HIP(hipGetLastError());
    return RSILU_OK;
}

rsilu_status_t rsilu_set_profiling(rsilu_handle_t h, int32_t enable)
{
    return rsilu_set_profiling_mask(h, enable ? (1u << RSILU_PROF_COUNT) - 1u : 0u);
}

rsilu_status_t rsilu_set_profiling_mask(rsilu_handle_t h, uint32_t mask)
{
    if (!h) return RSILU_EINVAL;
    if (mask >> RSILU_PROF_COUNT) return RSILU_EINVAL;
    h->prof_mask = mask;
    h->prof = mask != 0;
    h->ev_open.clear();
    h->ev_next = 0;
    for (int i = 0; i < RSILU_PROF_COUNT; ++i) {
        h->prof_launches[i] = 0;
        h->prof_ms[i] = 0.0;
        h->prof_bytes[i] = 0.0;
    }
    return RSILU_OK;
}

rsilu_status_t rsilu_get_profile(rsilu_handle_t h, rsilu_profile_t *out)
{
    if (!h || !out) return RSILU_EINVAL;
    for (int i = 0; i < RSILU_PROF_COUNT; ++i) {
        out->launches[i] = h->prof_launches[i];
        out->ms[i] = h->prof_ms[i];
        out->bytes[i] = h->prof_bytes[i];
    }
    return RSILU_OK;
}

void rsilu_destroy(rsilu_handle_t h)
{
    if (!h) return;
    release_graph(*h);
    if (h->cap_stream) (void)hipStreamDestroy(static_cast<hipStream_t>(h->cap_stream));
    if (h->pinned) (void)hipHostFree(h->pinned);
    for (void *e : h->ev_pool) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    delete h;
}

}  // extern "C"
