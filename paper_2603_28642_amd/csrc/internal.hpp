// Internal types shared by the host setup and the device driver.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "rsilu.h"
#include "level_rec.hpp"
#include "sweep_limits.hpp"

namespace rsilu {

// Host CSR with 32-bit row pointers (every operator has fewer than 2^31 entries).
struct Csr {
    int32_t nrows = 0, ncols = 0;
    std::vector<int32_t> ptr;  // nrows + 1
    std::vector<int32_t> col;
    std::vector<double> val;
    int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

// Level schedule of one triangular solve.
struct Levels {
    std::vector<int32_t> ptr;   // nlev + 1
    std::vector<int32_t> rows;  // n, rows ascending inside a level
    int32_t nlev() const { return ptr.empty() ? 0 : (int32_t)ptr.size() - 1; }
};

// Sync-free schedule: groups of consecutive rows of one level, each group at
// most `cap` rows, processed by one wavefront.
struct Chunks {
    std::vector<int32_t> ptr;  // nchunks + 1, positions in Levels::rows
    int32_t cap = 0;
};

// Hybrid schedule of a triangular solve. Levels wider than kSweepRows rows
// (or too large for the LDS) are separate multi-CU launches; runs of the other
// levels are swept by one workgroup, batch by batch: a batch is a contiguous
// byte blob (levels, rows, entries, diagonal) copied into LDS, and a row's
// input produced in the same batch is read from LDS.
struct Sweep {
    struct Seg {
        int32_t wide_level;  // >= 0: one multi-CU launch for this level
        int32_t b0, b1;      // otherwise: batches [b0, b1) in one single-workgroup launch
        int64_t rows, nnz;   // rows solved and stored entries read by the launch
        int32_t scheme;      // single-workgroup launch: its level scheme (kScheme*)
    };
    std::vector<Seg> segs;
    std::vector<int64_t> batch_off;  // nbatches + 1 byte offsets into blob
    std::vector<unsigned char> blob;
};

// A triangular factor with its rows stored in level order (position p holds
// row Levels::rows[p]); diag is the reciprocal of the diagonal in the same order
// (empty: unit).
// Read by the batched persistent solves: one load of the row pointer per
// position instead of the row index, then its pointer.
struct LoTri {
    Csr a;
    std::vector<double> diag;
    std::vector<unsigned char> rec;  // LevelRec<V> per position (V: the factor value type)
};

// Work plan for a CSR product: rows with more than `long_thresh` entries are
// split into segments of at most `seg` entries, reduced in a fixed order.
struct SpmvPlan {
    int32_t lanes = 8;           // lanes per row for ordinary rows
    int32_t unroll = 2;          // entries per lane loaded at once (paired-row kernel)
    int32_t long_thresh = 0;     // rows longer than this are "long"
    std::vector<int32_t> long_rows;
    std::vector<int32_t> seg_ptr;   // long row i owns segments seg_ptr[i]..seg_ptr[i+1]
    std::vector<int32_t> seg_beg;   // entry range of each segment
    std::vector<int32_t> seg_end;
};

// Offsets (bytes) of every array inside the caller's device buffer.
struct DevCsrOff {
    size_t ptr = 0, col = 0, val = 0;
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;
    int32_t vbytes = 8;  // 8: FP64 values, 4: FP32 (factors of the FP32 preconditioner)
};
struct DevPlanOff {
    size_t long_rows = 0, seg_ptr = 0, seg_beg = 0, seg_end = 0;
    int32_t nlong = 0, nseg = 0, lanes = 8, long_thresh = 0, unroll = 2;
};
struct DevTriOff {
    DevCsrOff a;
    size_t diag = 0;     // 0 = unit diagonal
    size_t rows = 0;     // level-ordered rows
    size_t chunk = 0;    // chunk pointer
    int32_t nchunks = 0;
    int32_t cap = 0;
    int32_t lanes = 8;
    int32_t nlev = 0;
    size_t blob = 0;  // hybrid sweep: batch blobs
    // level pointer and the level-ordered copy (LoTri) of the batched solves
    size_t lev = 0;
    DevCsrOff lo;
    size_t ldiag = 0;  // 0 = unit diagonal
    size_t lrec = 0;   // LevelRec per position
};

struct Layout {
    size_t total = 0;
    DevCsrOff A, AT, L2, L2T;
    DevPlanOff pA, pAT, pL2, pL2T;
    DevCsrOff Y, YT;     // explicit Y~ (rows in yperm order) and its transpose (RSILU_Y_EXPLICIT)
    DevPlanOff pY, pYT;
    size_t yperm = 0, yperm_inv = 0, yk = 0;  // the row order, its inverse, an (m-n)-vector
    DevTriOff L1f, L1b, Ub, UTf;  // L1 forward, L1^T backward, U backward, U^T forward
    size_t perm = 0, colnorm = 0, sfac = 0;
    // removed rows (present when R has rows): R, R^T, W's factor, and work vectors
    DevCsrOff R, RT;
    DevPlanOff pR, pRT;
    size_t wfac = 0, wr = 0, wz = 0, wh = 0;
    // Krylov vectors
    size_t xh = 0, p = 0, z = 0, h = 0, t = 0, y = 0, v = 0, g = 0, gp = 0, s2 = 0, c2 = 0;  // n
    size_t r = 0, q = 0;                                                       // m
    size_t u = 0;                                                              // m - n
    size_t lo_rhs = 0, lo_add = 0;  // level-ordered right-hand side and addend of a sweep (n)
    size_t f32a = 0, f32b = 0;      // FP32 preconditioner: converted input and output (m floats each)
    size_t cg_w = 0, cg_r = 0, cg_p = 0, cg_q = 0;  // CG or Chebyshev steps on S~ (m - n each)
    size_t cheb = 0;  // Chebyshev step coefficients c1[K] then c2[K] (read by the batched kernel)
    size_t cg_d = 0, cg_z = 0;  // Jacobi CG steps: diag(S~) and the preconditioned residual (m - n each)
    size_t cg_part = 0;  // CG steps: per-block partials of (p, q) and of two steps' (res, z), kCgParts each
    size_t l_v = 0, l_mv = 0, l_w = 0;              // LSQR: v, M v, w (n each)
    size_t partials = 0;  // reduction partials
    int32_t npartials = 0;
    size_t segpart = 0;   // long-row segment partials
    int32_t nsegpart = 0;
    size_t state = 0;     // device scalars and flags
};

struct Ctx {
    int64_t m = 0, n = 0, nnz_a = 0;
    rsilu_params_t prm{};
    int32_t smode = RSILU_S_IDENTITY;
    int64_t nmod = 0;

    std::vector<int32_t> perm;     // position -> original row
    std::vector<double> colnorm;   // n
    Csr A;                         // user's A (validated), original order, unscaled
    Csr Ahat, AhatT;               // pivot order, prescaled
    Csr L1, L1T, L2, L2T, U, UT;   // strictly triangular parts
    std::vector<double> Udiag;
    Levels lvL1, lvL1T, lvU, lvUT;
    Chunks chL1, chL1T, chU, chUT;
    Sweep swL1, swL1T, swU, swUT;
    LoTri loL1, loL1T, loU, loUT;
    SpmvPlan plA, plAT, plL2, plL2T;
    std::vector<double> sfac;      // packed lower Cholesky factor of S~ (dense mode)
    Csr Y, YT;                     // explicit Y~ = L2 L1^{-1} (Section 3.2) and its transpose
    Csr Yd, YdT;                   // the device copy: Y~'s rows in yperm order, and its transpose
    std::vector<int32_t> yperm, yperm_inv;  // device row i of Y~ is row yperm[i]
    SpmvPlan plY, plYT;            // plans of Yd and YdT
    // Chebyshev M_b (RSILU_S_CHEB): interval [1, cheb_b], cheb_K steps with coefficients
    // d <- c1[j] d + c2[j] r, starting from r = omega u, d = r / theta
    double cheb_b = 1.0, cheb_theta = 1.0, cheb_omega = 1.0;
    int32_t cheb_K = 0;
    std::vector<double> cheb_c1, cheb_c2;
    // Jacobi-preconditioned CG steps (RSILU_CG_JACOBI): diag(S~) in Y~'s device row order
    std::vector<double> cg_diag;
    // Section 3.4, removed rows: R = the removed rows of A_hat that were in A1, and the packed
    // lower Cholesky factor of W = I - R M^{-1} R^T (Woodbury update of the preconditioner)
    Csr R, RT;
    SpmvPlan plR, plRT;
    std::vector<double> wfac;

    Layout lay;
    // device side
    void *dev = nullptr;
    size_t dev_bytes = 0;
    int device = -1;
    void *pinned = nullptr;  // small host-pinned mailbox for polling
    void *graph_exec = nullptr;  // hipGraphExec_t of `poll` captured iterations (per upload)
    void *cap_stream = nullptr;  // hipStream_t the iterations are captured on

    // kernel timing (rsilu_set_profiling, rsilu_set_profiling_mask): prof is set when any
    // class is timed, prof_mask holds the timed classes (bit i: class i)
    bool prof = false;
    uint32_t prof_mask = 0;
    std::vector<void *> ev_pool;                // hipEvent_t
    struct EvRec {
        int cls, idx, iter;  // class, first of two events, iteration it belongs to (0 = init)
        double bytes;        // algorithmic bytes of the timed launch (kernel classes)
    };
    std::vector<EvRec> ev_open;                 // recorded, not yet read back
    int ev_iter = 0;                            // iteration being enqueued
    size_t ev_next = 0;
    int64_t prof_launches[RSILU_PROF_COUNT] = {};
    double prof_ms[RSILU_PROF_COUNT] = {};
    double prof_bytes[RSILU_PROF_COUNT] = {};
};

inline bool fp32(const Ctx &c) { return c.prm.precision == RSILU_PREC_FP32; }

// host setup (setup.cpp)
rsilu_status_t build_factorization(Ctx &c, int64_t m, int64_t n, const int64_t *rowptr,
                                   const int32_t *colind, const double *val);
void plan_layout(Ctx &c);
rsilu_status_t append_rows(Ctx &c, int64_t count, const int64_t *rowptr, const int32_t *colind, const double *val);
rsilu_status_t remove_rows(Ctx &c, int64_t count, const int64_t *rows);
rsilu_status_t build_woodbury(Ctx &c);
void build_explicit_Y(Ctx &c);
void build_chebyshev(Ctx &c);
inline bool yexplicit(const Ctx &c) { return c.prm.ystore == RSILU_Y_EXPLICIT; }
// device driver (capi.hip): drop a captured iteration graph
void release_graph(Ctx &c);

}  // namespace rsilu

// The opaque handle of the C ABI (rsilu.h) is the context itself.
struct rsilu_ctx : rsilu::Ctx {};
