// C ABI of the library and the device driver of the solve (Algorithm 1 with
// Algorithm 3 or Algorithm 2), enqueued on the caller's stream. The host only enqueues work
// and polls a stop flag every `poll` iterations; every scalar of the
// recurrence lives on the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "kernels.hpp"

struct rsilu_ctx : rsilu::Ctx {};

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
                 at<int32_t>(c, o.seg_end), o.nlong, o.nseg, o.lanes, o.long_thresh};
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
        if (!c_.prof) return;
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
    DPlan pA, pAT, pL2, pL2T;
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

// One triangular solve with the configured schedule. Sync-free solves need x
// sentinel-filled and their ticket cleared beforehand.
void trsv(Ctx &c, hipStream_t s, const Ptrs &P, const DTri &t, const Levels &lv, const Sweep &sw,
          const DevTriOff &o, const double *rhs, double *x, const double *add, double *y2, int ticket,
          const int32_t *done, int cls)
{
    ProfScope ps(c, s, cls);
    if (c.prm.trsv == RSILU_TRSV_HYBRID) {
        const unsigned char *blob = at<unsigned char>(c, o.blob);
        const bool runs = std::any_of(sw.segs.begin(), sw.segs.end(), [](const Sweep::Seg &g) { return g.wide_level < 0; });
        // algorithmic bytes of a launch solving `rows` rows with `nnz` stored entries:
        // values and column indices once, per row its pointer, level-list entry,
        // right-hand side and result (plus diagonal, fused addend and sum)
        const double per_row = 24.0 + (t.diag ? 8.0 : 0.0) + (y2 ? 16.0 : 0.0);
        auto bytes = [&](int64_t rows, int64_t nnz) { return 12.0 * (double)nnz + per_row * (double)rows; };
        if (runs) {
            ProfScope pg(c, s, RSILU_PROF_K_GATHER, (double)c.n * (y2 ? 36.0 : 20.0));
            launch_gather_lo(s, (int32_t)c.n, t.rows, rhs, P.lo_rhs, add, y2 ? P.lo_add : nullptr, done);
        }
        for (const Sweep::Seg &g : sw.segs) {
            if (g.wide_level >= 0) {
                ProfScope pk(c, s, RSILU_PROF_K_LEVEL, bytes(g.rows, g.nnz));
                launch_trsv_level(s, t, lv.ptr[g.wide_level], lv.ptr[(size_t)g.wide_level + 1], rhs, x, add, y2,
                                  done);
            } else {
                const int64_t off = sw.batch_off[(size_t)g.b0];
                const int32_t size = (int32_t)(sw.batch_off[(size_t)g.b0 + 1] - off);
                const int32_t *h0 = reinterpret_cast<const int32_t *>(sw.blob.data() + off);
                ProfScope pk(c, s, RSILU_PROF_K_SWEEP, bytes(g.rows, g.nnz));
                launch_trsv_sweep(s, blob, off, size, h0[1], h0[6], g.b1 - g.b0, P.lo_rhs, x, P.lo_add, y2, done);
            }
        }
    } else if (c.prm.trsv == RSILU_TRSV_LEVELS) {
        for (int32_t l = 0; l < lv.nlev(); ++l)
            launch_trsv_level(s, t, lv.ptr[l], lv.ptr[(size_t)l + 1], rhs, x, add, y2, done);
    } else {
        launch_trsv_syncfree(s, t, rhs, x, add, y2, P.st, ticket, done);
    }
}

bool syncfree(const Ctx &c) { return c.prm.trsv == RSILU_TRSV_SYNCFREE; }

// Algorithm 3 on the residual r (pivot order) -> hout. For sync-free solves the
// outputs t, gp, v and hout must have been sentinel-filled, tickets cleared.
void apply_alg3(Ctx &c, hipStream_t s, const Ptrs &P, const double *r, double *hout, const int32_t *done)
{
    const int32_t n = (int32_t)c.n, k = (int32_t)(c.m - c.n);
    // step 1: u = r2 - Y r1 with Y r1 = L2 (L1^{-1} r1)
    trsv(c, s, P, P.L1f, c.lvL1, c.swL1, c.lay.L1f, r, P.t, nullptr, nullptr, 0, done, RSILU_PROF_TRSV_L1);
    if (k == 0 || c.smode == RSILU_S_NONE) {
        // no A2 or no correction (w = 0): h = U^{-1} L1^{-1} r1
        trsv(c, s, P, P.Ub, c.lvU, c.swU, c.lay.Ub, P.t, hout, nullptr, nullptr, 3, done, RSILU_PROF_TRSV_U);
        return;
    }
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_L2);
        launch_spmv(s, P.L2, P.pL2, P.t, P.u, r + n, EPI_SUB, FIN_NONE, P.partials, P.segpart, P.st, done);
    }
    // step 2: S^ w = u (in place in u)
    if (c.smode == RSILU_S_DENSE) {
        ProfScope ps(c, s, RSILU_PROF_DENSE_S);
        launch_dense_chol_solve(s, k, P.sfac, P.u, done);
    }
    // step 3: y = r1 + Y^T w with Y^T w = L1^{-T} (L2^T w)
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_L2T);
        launch_spmv(s, P.L2T, P.pL2T, P.u, P.g, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, done);
    }
    trsv(c, s, P, P.L1b, c.lvL1T, c.swL1T, c.lay.L1b, P.g, P.gp, r, P.y, 1, done, RSILU_PROF_TRSV_L1T);
    // step 4: L1 v = y, U h = v
    trsv(c, s, P, P.L1f, c.lvL1, c.swL1, c.lay.L1f, P.y, P.v, nullptr, nullptr, 2, done, RSILU_PROF_TRSV_L1);
    trsv(c, s, P, P.Ub, c.lvU, c.swU, c.lay.Ub, P.v, hout, nullptr, nullptr, 3, done, RSILU_PROF_TRSV_U);
}

// Whether Algorithm 2 carries the M_b correction (six triangular sweeps
// instead of four).
bool alg2_correction(const Ctx &c) { return c.m > c.n && c.smode != RSILU_S_NONE; }

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
void apply_alg2(Ctx &c, hipStream_t s, const Ptrs &P, const double *z, double *hout, const int32_t *done)
{
    const int32_t n = (int32_t)c.n, k = (int32_t)(c.m - c.n);
    trsv(c, s, P, P.UTf, c.lvUT, c.swUT, c.lay.UTf, z, P.t, nullptr, nullptr, 0, done, RSILU_PROF_TRSV_UT);
    trsv(c, s, P, P.L1b, c.lvL1T, c.swL1T, c.lay.L1b, P.t, P.gp, nullptr, nullptr, 1, done, RSILU_PROF_TRSV_L1T);
    if (!alg2_correction(c)) {
        trsv(c, s, P, P.L1f, c.lvL1, c.swL1, c.lay.L1f, P.gp, P.v, nullptr, nullptr, 2, done, RSILU_PROF_TRSV_L1);
        trsv(c, s, P, P.Ub, c.lvU, c.swU, c.lay.Ub, P.v, hout, nullptr, nullptr, 3, done, RSILU_PROF_TRSV_U);
        return;
    }
    // step 2: w_b = L2 (L1^{-1} g) into u
    trsv(c, s, P, P.L1f, c.lvL1, c.swL1, c.lay.L1f, P.gp, P.v, nullptr, nullptr, 2, done, RSILU_PROF_TRSV_L1);
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_L2);
        launch_spmv(s, P.L2, P.pL2, P.v, P.u, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, done);
    }
    // step 3: v_b = M_b^{-1} w_b in place
    if (c.smode == RSILU_S_DENSE) {
        ProfScope ps(c, s, RSILU_PROF_DENSE_S);
        launch_dense_chol_solve(s, k, P.sfac, P.u, done);
    }
    // steps 4-5: y = g + L1^{-T} (-L2^T v_b), then L1 s2 = y, U h = s2
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_L2T);
        launch_spmv(s, P.L2T, P.pL2T, P.u, P.g, nullptr, EPI_NEG, FIN_NONE, P.partials, P.segpart, P.st, done);
    }
    trsv(c, s, P, P.L1b, c.lvL1T, c.swL1T, c.lay.L1b, P.g, P.c2, P.gp, P.y, 3, done, RSILU_PROF_TRSV_L1T);
    if (syncfree(c)) launch_refill(s, n, P.s2, hout, P.st, done);
    trsv(c, s, P, P.L1f, c.lvL1, c.swL1, c.lay.L1f, P.y, P.s2, nullptr, nullptr, 0, done, RSILU_PROF_TRSV_L1);
    trsv(c, s, P, P.Ub, c.lvU, c.swU, c.lay.Ub, P.s2, hout, nullptr, nullptr, 1, done, RSILU_PROF_TRSV_U);
}

void apply_form(Ctx &c, hipStream_t s, const Ptrs &P, double *hout, const int32_t *done)
{
    if (c.prm.form == RSILU_FORM_ALG2)
        apply_alg2(c, s, P, P.z, hout, done);
    else
        apply_alg3(c, s, P, P.r, hout, done);
}

void enqueue_iteration(Ctx &c, hipStream_t s, const Ptrs &P)
{
    const int32_t n = (int32_t)c.n, m = (int32_t)c.m;
    // q = A p, alpha = rho / (q, q)
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_A);
        launch_spmv(s, P.A, P.pA, P.p, P.q, nullptr, EPI_SQ, FIN_ALPHA, P.partials, P.segpart, P.st, P.done);
    }
    // x += alpha p, r -= alpha q (and prepare the sync-free outputs)
    const bool sf = syncfree(c);
    double *f[4];
    fill_targets(c, P, P.h, f);
    launch_update(s, n, m, P.p, P.xh, P.q, P.r, sf ? f[0] : nullptr, f[1], f[2], f[3], P.st, P.done);
    // z = A^T r, stop test on ||D^{-1} z|| = ||A^T r||
    {
        ProfScope ps(c, s, RSILU_PROF_SPMV_AT);
        launch_spmv(s, P.AT, P.pAT, P.r, P.z, P.colnorm, EPI_WSQ, FIN_STOP, P.partials, P.segpart, P.st, P.done);
    }
    // h = M^{-1} z by Algorithm 3 on (r1, r2) or Algorithm 2 on z
    apply_form(c, s, P, P.h, P.done);
    // rho' = (z, h), beta = rho'/rho, p = h + beta p
    launch_dot(s, n, P.z, P.h, FIN_BETA, P.partials, P.st, P.done);
    launch_pupdate(s, n, P.h, P.p, P.st, false, P.done);
}

}  // namespace
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
    const int64_t k = h->m - h->n;
    s->psize = s->nnz_l1 + s->nnz_l2 + s->nnz_u + h->n + (h->smode == RSILU_S_DENSE ? k * (k + 1) / 2 : 0);
    s->nmod = h->nmod;
    s->levels_l1 = h->lvL1.nlev();
    s->levels_l1t = h->lvL1T.nlev();
    s->levels_u = h->lvU.nlev();
    s->levels_ut = h->lvUT.nlev();
    s->smode = h->smode;
    s->device_bytes = h->lay.total;
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
    auto put_csr = [&](const DevCsrOff &o, const Csr &a) -> hipError_t {
        hipError_t e = put(o.ptr, a.ptr.data(), a.ptr.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.col, a.col.data(), a.col.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.val, a.val.data(), a.val.size() * sizeof(double));
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
                       const Chunks &ch) -> hipError_t {
        hipError_t e = put_csr(o.a, a);
        if (e == hipSuccess && diag) e = put(o.diag, diag->data(), diag->size() * sizeof(double));
        if (e == hipSuccess) e = put(o.rows, lv.rows.data(), lv.rows.size() * sizeof(int32_t));
        if (e == hipSuccess) e = put(o.chunk, ch.ptr.data(), ch.ptr.size() * sizeof(int32_t));
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
    RSILU_HIP(put_tri(L.L1f, c.L1, nullptr, c.lvL1, c.chL1));
    RSILU_HIP(put_tri(L.L1b, c.L1T, nullptr, c.lvL1T, c.chL1T));
    RSILU_HIP(put_tri(L.Ub, c.U, &c.Udiag, c.lvU, c.chU));
    RSILU_HIP(put_tri(L.UTf, c.UT, &c.Udiag, c.lvUT, c.chUT));
    RSILU_HIP(put_sweep(L.L1f, c.swL1));
    RSILU_HIP(put_sweep(L.L1b, c.swL1T));
    RSILU_HIP(put_sweep(L.Ub, c.swU));
    RSILU_HIP(put_sweep(L.UTf, c.swUT));
    RSILU_HIP(put(L.perm, c.perm.data(), c.perm.size() * sizeof(int32_t)));
    RSILU_HIP(put(L.colnorm, c.colnorm.data(), c.colnorm.size() * sizeof(double)));
    RSILU_HIP(put(L.sfac, c.sfac.data(), c.sfac.size() * sizeof(double)));
    PinnedMail *mail = static_cast<PinnedMail *>(c.pinned);
    std::memset(&mail->init, 0, sizeof(DevState));
    RSILU_HIP(hipMemcpyAsync(at<DevState>(c, L.state), &mail->init, sizeof(DevState), hipMemcpyHostToDevice, s));
    RSILU_HIP(hipStreamSynchronize(s));
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

    // ---- initialisation: x0 = 0, r0 = P b, z0 = A^T r0, h0 = B(r0), rho0, p0 = h0
    c.ev_iter = 0;
    c.ev_open.clear();
    c.ev_next = 0;
    launch_gather(s, m, n, P.perm, b, P.r, P.xh, nullptr);
    launch_spmv(s, P.AT, P.pAT, P.r, P.z, P.colnorm, EPI_WSQ, FIN_INIT, P.partials, P.segpart, P.st, nullptr);
    if (sf) {
        double *f[4];
        fill_targets(c, P, P.h, f);
        launch_fill(s, n, f[0], f[1], f[2], f[3], P.st);
    }
    apply_form(c, s, P, P.h, P.done);
    launch_dot(s, n, P.z, P.h, FIN_RHO0, P.partials, P.st, P.done);
    launch_pupdate(s, n, P.h, P.p, P.st, true, P.done);
    RSILU_HIP(hipGetLastError());

    // ---- iterations, polled every `poll` steps (maxit = 0 stops after the init)
    int64_t enqueued = 0;
    bool stop = c.prm.maxit == 0;
    while (!stop) {
        const int batch = (int)std::min<int64_t>(c.prm.poll, (int64_t)c.prm.maxit - enqueued);
        for (int i = 0; i < batch; ++i) {
            c.ev_iter = (int)(enqueued + i + 1);
            enqueue_iteration(c, s, P);
        }
        enqueued += batch;
        RSILU_HIP(hipGetLastError());
        RSILU_HIP(hipMemcpyAsync(&mail->poll, P.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        RSILU_HIP(hipStreamSynchronize(s));
        if (c.prof) prof_collect(c, mail->poll.done ? mail->poll.iter - 1 : mail->poll.iter);
        if (mail->poll.done || mail->poll.err || enqueued >= c.prm.maxit) stop = true;
    }

    // ---- exit: x = D x_hat; true ||A^T (b - A x)|| recomputed from x_hat
    launch_scale_out(s, n, P.xh, P.colnorm, x);
    launch_spmv(s, P.A, P.pA, P.xh, P.q, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, nullptr);
    launch_residual(s, m, P.perm, b, P.q, P.r);
    launch_spmv(s, P.AT, P.pAT, P.r, P.z, P.colnorm, EPI_WSQ, FIN_ATR, P.partials, P.segpart, P.st, nullptr);
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
    const Ptrs P = ptrs(*h);
    switch (op) {
    case 0: launch_spmv(s, P.A, P.pA, xin, y, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, nullptr); break;
    case 1: launch_spmv(s, P.AT, P.pAT, xin, y, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, nullptr); break;
    case 2: launch_spmv(s, P.L2, P.pL2, xin, y, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, nullptr); break;
    case 3: launch_spmv(s, P.L2T, P.pL2T, xin, y, nullptr, EPI_PLAIN, FIN_NONE, P.partials, P.segpart, P.st, nullptr); break;
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
    Ctx &c = *h;
    const Ptrs P = ptrs(c);
    const int32_t n = (int32_t)c.n;
    if (syncfree(c)) launch_fill(s, n, x, nullptr, nullptr, nullptr, P.st);
    switch (which) {
    case 0: trsv(c, s, P, P.L1f, c.lvL1, c.swL1, c.lay.L1f, rhs, x, nullptr, nullptr, 0, nullptr, RSILU_PROF_TRSV_L1); break;
    case 1: trsv(c, s, P, P.L1b, c.lvL1T, c.swL1T, c.lay.L1b, rhs, x, nullptr, nullptr, 0, nullptr, RSILU_PROF_TRSV_L1T); break;
    case 2: trsv(c, s, P, P.Ub, c.lvU, c.swU, c.lay.Ub, rhs, x, nullptr, nullptr, 0, nullptr, RSILU_PROF_TRSV_U); break;
    case 3: trsv(c, s, P, P.UTf, c.lvUT, c.swUT, c.lay.UTf, rhs, x, nullptr, nullptr, 0, nullptr, RSILU_PROF_TRSV_UT); break;
    default: return RSILU_EINVAL;
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
    if (syncfree(c)) launch_fill(s, (int32_t)c.n, P.t, P.gp, P.v, hout, P.st);
    apply_alg3(c, s, P, r, hout, nullptr);
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
    if (syncfree(c)) launch_fill(s, (int32_t)c.n, P.t, P.gp, P.v, alg2_correction(c) ? P.c2 : hout, P.st);
    apply_alg2(c, s, P, z, hout, nullptr);
    RSILU_HIP(hipGetLastError());
    return RSILU_OK;
}

rsilu_status_t rsilu_set_profiling(rsilu_handle_t h, int32_t enable)
{
    if (!h) return RSILU_EINVAL;
    h->prof = enable != 0;
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
    if (h->pinned) (void)hipHostFree(h->pinned);
    for (void *e : h->ev_pool) (void)hipEventDestroy(static_cast<hipEvent_t>(e));
    delete h;
}

}  // extern "C"
