// Host setup of the row-splitting ILU preconditioner.
//
//   validate     CSR input of A, explicit zeros stripped            (1.1)
//   prescale     unit 2-norm columns                                Section 5.1
//   ilup         rectangular ILUP(p, tau), threshold partial
//                pivoting by rows, minimum row count, modification  Algorithms 4-6
//   split        P A D ~ [L1; L2] U, transposes                     (3.8)
//   levels       dependency levels of the triangular solves
//   dense S~     S~ = I + Y Y^T, Y = L2 L1^{-1}, Cholesky           Section 3.2
//   explicit Y~  Y~ = L2 L1^{-1} as a sparse matrix, small entries
//                dropped                                            Section 3.2
//
// Floating-point decisions of the factorization (pivot choice, dropping) are
// taken on values computed in a fixed order with separately rounded products
// and sums (this file is compiled with -ffp-contract=off), so the row
// permutation and the factors are reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <queue>
#include <stdexcept>
#include <thread>
#include <utility>

#include "internal.hpp"

namespace rsilu {

namespace {

constexpr int64_t kMaxIdx = 2147483647LL;

// ---------------------------------------------------------------- CSR helpers

// Transpose of a CSR (counting sort by column; rows ascend within each output row).
Csr transpose(const Csr &a)
{
    Csr t;
    t.nrows = a.ncols;
    t.ncols = a.nrows;
    t.ptr.assign((size_t)t.nrows + 1, 0);
    for (int32_t c : a.col) t.ptr[(size_t)c + 1]++;
    for (int32_t i = 0; i < t.nrows; ++i) t.ptr[(size_t)i + 1] += t.ptr[i];
    t.col.resize(a.col.size());
    t.val.resize(a.val.size());
    std::vector<int32_t> fill(t.ptr.begin(), t.ptr.end() - 1);
    for (int32_t i = 0; i < a.nrows; ++i) {
        for (int32_t e = a.ptr[i]; e < a.ptr[(size_t)i + 1]; ++e) {
            int32_t d = fill[a.col[e]]++;
            t.col[d] = i;
            t.val[d] = a.val[e];
        }
    }
    return t;
}

// CSR from per-row (col, val) lists; each row is sorted by column.
Csr from_rows(int32_t nrows, int32_t ncols, std::vector<std::vector<std::pair<int32_t, double>>> &rows)
{
    Csr a;
    a.nrows = nrows;
    a.ncols = ncols;
    a.ptr.assign((size_t)nrows + 1, 0);
    for (int32_t i = 0; i < nrows; ++i) a.ptr[(size_t)i + 1] = a.ptr[i] + (int32_t)rows[i].size();
    a.col.reserve((size_t)a.ptr.back());
    a.val.reserve((size_t)a.ptr.back());
    for (auto &r : rows) {
        std::sort(r.begin(), r.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
        for (auto &e : r) {
            a.col.push_back(e.first);
            a.val.push_back(e.second);
        }
        std::vector<std::pair<int32_t, double>>().swap(r);
    }
    return a;
}

// ---------------------------------------------------------------- levels

// Kahn layering: a row becomes ready once all rows it depends on are placed;
// rows made ready by the same layer form the next level (sorted ascending).
// deps: row -> rows it reads; users: row -> rows that read it.
Levels kahn_levels(const Csr &deps, const Csr &users)
{
    const int32_t n = deps.nrows;
    Levels out;
    std::vector<int32_t> waiting((size_t)n);
    std::vector<int32_t> cur, next;
    for (int32_t i = 0; i < n; ++i) {
        waiting[i] = deps.ptr[(size_t)i + 1] - deps.ptr[i];
        if (waiting[i] == 0) cur.push_back(i);
    }
    out.rows.reserve((size_t)n);
    out.ptr.push_back(0);
    while (!cur.empty()) {
        std::sort(cur.begin(), cur.end());
        out.rows.insert(out.rows.end(), cur.begin(), cur.end());
        out.ptr.push_back((int32_t)out.rows.size());
        next.clear();
        for (int32_t r : cur)
            for (int32_t e = users.ptr[r]; e < users.ptr[(size_t)r + 1]; ++e)
                if (--waiting[users.col[e]] == 0) next.push_back(users.col[e]);
        cur.swap(next);
    }
    return out;
}

Chunks make_chunks(const Levels &lv, int32_t cap)
{
    Chunks ch;
    ch.cap = cap;
    ch.ptr.push_back(0);
    for (int32_t l = 0; l < lv.nlev(); ++l)
        for (int32_t s = lv.ptr[l]; s < lv.ptr[(size_t)l + 1]; s += cap)
            ch.ptr.push_back(std::min(s + cap, lv.ptr[(size_t)l + 1]));
    return ch;
}

// Byte offsets inside a sweep batch blob (layout in kernels.hip, k_trsv_sweep).
struct BlobLayout {
    int64_t lev, lch, row, ext, next_ext, rch, slot, val, diag, crow, size;
};
BlobLayout blob_layout(int64_t nlev, int64_t npos, int64_t next, int64_t nchunk, bool diag, int64_t vb, bool seg)
{
    BlobLayout o;
    o.lev = 4 * kSweepHdr;
    o.lch = o.lev + 4 * (nlev + 1);
    o.row = o.lch + 4 * (nlev + 1);
    o.ext = o.row + 4 * npos;
    o.next_ext = o.ext + 4 * next;
    o.rch = o.next_ext + 4 * (int64_t)kSweepExt;
    o.slot = (o.rch + 2 * (npos + 1) + 7) & ~(int64_t)7;
    o.val = (o.slot + 8 * nchunk + 15) & ~(int64_t)15;
    o.diag = o.val + 4 * vb * nchunk;
    o.crow = o.diag + (diag ? vb * npos : 0);
    o.size = (o.crow + (seg ? 2 * nchunk : 0) + 15) & ~(int64_t)15;
    return o;
}
int64_t blob_bytes(int64_t nlev, int64_t npos, int64_t next, int64_t nchunk, bool diag, int64_t vb, bool seg)
{
    return blob_layout(nlev, npos, next, nchunk, diag, vb, seg).size;
}

template <class V>
LoTri level_ordered(const Csr &T, const std::vector<double> *diag, const Levels &lv)
{
    LoTri o;
    const int32_t n = T.nrows;
    o.a.nrows = n;
    o.a.ncols = T.ncols;
    o.a.ptr.assign((size_t)n + 1, 0);
    o.a.col.reserve(T.col.size());
    o.a.val.reserve(T.val.size());
    if (diag) o.diag.resize((size_t)n);
    for (int32_t p = 0; p < n; ++p) {
        const int32_t row = lv.rows[p];
        for (int32_t e = T.ptr[row]; e < T.ptr[(size_t)row + 1]; ++e) {
            o.a.col.push_back(T.col[e]);
            o.a.val.push_back(T.val[e]);
        }
        o.a.ptr[(size_t)p + 1] = (int32_t)o.a.col.size();
        if (diag) o.diag[p] = 1.0 / (*diag)[row];  // reciprocal: the batched solves multiply
    }
    o.rec.assign(sizeof(LevelRec<V>) * (size_t)n, 0);
    LevelRec<V> *rec = reinterpret_cast<LevelRec<V> *>(o.rec.data());
    for (int32_t p = 0; p < n; ++p) {
        LevelRec<V> &r = rec[p];
        r.row = lv.rows[p];
        r.k0 = o.a.ptr[p];
        r.k1 = o.a.ptr[(size_t)p + 1];
        for (int j = 0; j < kRecEntries; ++j) {
            const bool in = r.k0 + j < r.k1;
            r.col[j] = in ? o.a.col[(size_t)r.k0 + j] : -1;
            r.val[j] = in ? (V)o.a.val[(size_t)r.k0 + j] : (V)0;
        }
        r.rdiag = diag ? (V)o.diag[p] : (V)1;
    }
    return o;
}

int64_t chunks_of(int64_t len) { return (len + kSweepChunk - 1) / kSweepChunk; }

// Hybrid sweep schedule of the triangular operator T with level sets lv.
// Runs of levels of at most kSweepRows rows are cut into batches; an input of a
// row is read from LDS: from the results of the same batch, of the previous
// batch of the run, or from the batch's gathered older inputs ("ext"). Rows
// are cut into chunks of at most kSweepChunk entries. In the segmented scheme a
// level's chunks are padded so no row of up to 16 chunks crosses a 16-chunk group
// and no longer row crosses a 64-chunk group, and a row without entries gets one
// chunk of padding (its lane solves it).
// V is the value type stored in the blob: double, or float for the FP32
// preconditioner (values rounded to nearest).
template <class V>
Sweep make_sweep(const Csr &T, const std::vector<double> *diag, const Levels &lv, int32_t force)
{
    constexpr int64_t vb = (int64_t)sizeof(V);
    Sweep sw;
    const int32_t n = T.nrows;
    const bool hd = diag != nullptr;
    std::vector<int32_t> posof((size_t)n);
    for (int32_t p = 0; p < n; ++p) posof[lv.rows[p]] = p;
    std::vector<int32_t> ext_stamp((size_t)n, -1), ext_slot((size_t)n, 0);
    sw.batch_off.push_back(0);
    auto nbatches = [&]() { return (int32_t)sw.batch_off.size() - 1; };
    auto rowlen = [&](int32_t row) { return (int64_t)T.ptr[(size_t)row + 1] - T.ptr[row]; };
    auto entries = [&](int32_t l) {
        int64_t ne = 0;
        for (int32_t p = lv.ptr[l]; p < lv.ptr[(size_t)l + 1]; ++p) ne += rowlen(lv.rows[p]);
        return ne;
    };
    auto maxchunks = [&](int32_t l) {
        int64_t mx = 0;
        for (int32_t p = lv.ptr[l]; p < lv.ptr[(size_t)l + 1]; ++p) mx = std::max(mx, chunks_of(rowlen(lv.rows[p])));
        return mx;
    };
    // Level scheme of the whole factor, from its narrow levels' longest rows (measured
    // on gfx950): when nearly every level's rows have at most 64 chunks, a row's chunks
    // on consecutive lanes of one 16-lane DPP row (rows of more than 16 chunks: of one
    // wavefront), summed by a segmented scan (kSchemeSegmented, or kSchemeSegmentedWide
    // when some row has more than 16 chunks; a level with a row of more than 64 becomes
    // a wide level); else two phases per level (chunk sums, then row sums). The
    // one-row-per-thread scheme is selected only on request.
    int32_t scheme;
    bool over16 = false;  // a narrow level holds a row of 17..64 chunks
    {
        int64_t nl = 0, le64 = 0;
        for (int32_t l = 0; l < lv.nlev(); ++l) {
            if (lv.ptr[(size_t)l + 1] - lv.ptr[l] > kSweepRows) continue;
            const int64_t mx = maxchunks(l);
            ++nl;
            le64 += mx <= 64 ? 1 : 0;
            over16 = over16 || (mx > 16 && mx <= 64);
        }
        scheme = le64 >= 0.95 * (double)nl ? kSchemeSegmented : kSchemeTwoPhase;
        if (force == RSILU_SWEEP_TWO_PHASE) scheme = kSchemeTwoPhase;
        if (force == RSILU_SWEEP_SEGMENTED) scheme = kSchemeSegmented;
        if (force == RSILU_SWEEP_ROWS) scheme = kSchemeRows;
    }
    // rows of more than 16 chunks need the wavefront-wide scan (its own instantiation,
    // so factors without such rows run the 16-lane one)
    if (scheme == kSchemeSegmented && over16) scheme = kSchemeSegmentedWide;
    const bool seg = scheme == kSchemeSegmented || scheme == kSchemeSegmentedWide;
    // chunks of a row in the blob: in the segmented scheme a row without entries still
    // gets one (its lane solves it)
    auto rchunks = [&](int32_t row) { return seg ? std::max<int64_t>(1, chunks_of(rowlen(row))) : chunks_of(rowlen(row)); };
    // lanes a row of k chunks must not cross in the segmented scheme: one 16-lane group,
    // or the wavefront for rows of more than 16 chunks
    auto group_of = [](int64_t k) -> int64_t { return k <= 16 ? 16 : 64; };
    // chunk count of level l, with the padding that keeps each row inside its group
    auto chunks = [&](int32_t l) {
        int64_t nc = 0;
        for (int32_t p = lv.ptr[l]; p < lv.ptr[(size_t)l + 1]; ++p) {
            const int64_t k = rchunks(lv.rows[p]), g = group_of(k);
            if (seg && (nc % g) + k > g) nc += g - nc % g;
            nc += k;
        }
        return nc;
    };

    int32_t run_b0 = -1;                 // first batch of the open run
    int32_t prev_p0 = -1, prev_p1 = -1;  // positions of the previous batch of the run
    int32_t bl0 = -1, bl1 = -1;          // levels of the open batch
    int64_t bpos = 0, bent = 0, bchk = 0;
    int32_t stamp = 0;
    std::vector<int64_t> batch_rows, batch_nnz;  // per serialized batch

    // older inputs of level l that a batch starting at position p0 would gather
    auto new_ext = [&](int32_t l, int32_t p0) {
        int64_t k = 0;
        for (int32_t p = lv.ptr[l]; p < lv.ptr[(size_t)l + 1]; ++p) {
            const int32_t row = lv.rows[p];
            for (int32_t e = T.ptr[row]; e < T.ptr[(size_t)row + 1]; ++e) {
                const int32_t c = T.col[e], pc = posof[c];
                if (pc >= p0 || (pc >= prev_p0 && pc < prev_p1)) continue;
                if (ext_stamp[c] != stamp) {
                    ext_stamp[c] = stamp;
                    ++k;
                }
            }
        }
        return k;
    };

    auto serialize = [&](int32_t l0, int32_t l1) {
        const int32_t p0 = lv.ptr[l0], p1 = lv.ptr[l1], npos = p1 - p0, nlev = l1 - l0;
        const int32_t bi = nbatches() - run_b0;  // index inside the run
        const int32_t cur_base = (bi & 1) ? kSweepPos : 0, prev_base = (bi & 1) ? 0 : kSweepPos;
        ++stamp;
        std::vector<int32_t> ext;
        int64_t nent = 0, nchunk = 0;
        for (int32_t l = l0; l < l1; ++l) nchunk += chunks(l);
        for (int32_t p = p0; p < p1; ++p) {
            const int32_t row = lv.rows[p];
            for (int32_t e = T.ptr[row]; e < T.ptr[(size_t)row + 1]; ++e, ++nent) {
                const int32_t c = T.col[e], pc = posof[c];
                if (pc >= p0 || (pc >= prev_p0 && pc < prev_p1)) continue;
                if (ext_stamp[c] != stamp) {
                    ext_stamp[c] = stamp;
                    ext_slot[c] = (int32_t)ext.size();
                    ext.push_back(c);
                }
            }
        }
        const int64_t next = (int64_t)ext.size();
        const BlobLayout lay = blob_layout(nlev, npos, next, nchunk, hd, vb, seg);
        const int64_t size = lay.size;
        if (npos > kSweepPos || next > kSweepExt || size > kSweepBlob || nchunk > 65535 || nlev > kSweepLevels)
            throw std::length_error("sweep batch exceeds the LDS limits");
        const size_t base = sw.blob.size();
        sw.blob.resize(base + (size_t)size, 0);
        unsigned char *b = sw.blob.data() + base;
        int32_t *hdr = reinterpret_cast<int32_t *>(b);
        hdr[0] = nlev;
        hdr[1] = npos;
        hdr[2] = (int32_t)(kSweepChunk * nchunk);
        hdr[3] = (int32_t)next;
        hdr[4] = hd ? 1 : 0;
        hdr[5] = cur_base;
        hdr[6] = p0;
        hdr[7] = (int32_t)size;
        hdr[8] = 0;   // size of the next batch of the run (patched by the next batch)
        hdr[9] = 0;   // rows of the next batch
        hdr[10] = 0;  // older inputs of the next batch (their rows follow ext_idx)
        hdr[11] = (int32_t)nchunk;
        int32_t *lev_off = reinterpret_cast<int32_t *>(b + lay.lev);
        int32_t *lev_chunk = reinterpret_cast<int32_t *>(b + lay.lch);
        int32_t *rowid = reinterpret_cast<int32_t *>(b + lay.row);
        int32_t *ext_idx = reinterpret_cast<int32_t *>(b + lay.ext);
        uint16_t *rchunk = reinterpret_cast<uint16_t *>(b + lay.rch);
        uint16_t *eslot = reinterpret_cast<uint16_t *>(b + lay.slot);
        V *eval = reinterpret_cast<V *>(b + lay.val);
        V *dg = reinterpret_cast<V *>(b + lay.diag);
        uint16_t *crow = reinterpret_cast<uint16_t *>(b + lay.crow);  // segmented scheme only
        for (int64_t j = 0; j < next; ++j) ext_idx[j] = ext[(size_t)j];
        int32_t ch = 0;
        int32_t lvl = l0;
        lev_off[0] = 0;
        lev_chunk[0] = 0;
        auto pad_chunk = [&](uint16_t who) {
            for (int32_t q = 0; q < kSweepChunk; ++q) {
                eslot[(int64_t)kSweepChunk * ch + q] = (uint16_t)kSweepZeroSlot;
                eval[(int64_t)kSweepChunk * ch + q] = (V)0;
            }
            crow[ch] = who;
            ++ch;
        };
        int32_t lch0 = 0;  // first chunk of the current level
        for (int32_t p = p0; p < p1; ++p) {
            while (p >= lv.ptr[(size_t)lvl + 1]) {
                ++lvl;
                lev_off[lvl - l0] = p - p0;
                lev_chunk[lvl - l0] = ch;
                lch0 = ch;
            }
            const int32_t row = lv.rows[p];
            rowid[p - p0] = row;
            if (seg) {
                // keep the row's chunks inside its group of the level's lanes
                const int64_t k = rchunks(row), t = ch - lch0, g = group_of(k);
                if ((t % g) + k > g)
                    for (int64_t q = t % g; q < g; ++q) pad_chunk(0x7fff);
                if (rowlen(row) == 0) {
                    rchunk[p - p0] = (uint16_t)ch;
                    pad_chunk((uint16_t)(0x8000 | (p - p0)));
                    if (hd) dg[p - p0] = (V)(1.0 / (*diag)[row]);
                    continue;
                }
            }
            rchunk[p - p0] = (uint16_t)ch;
            int32_t k = T.ptr[row];
            while (k < T.ptr[(size_t)row + 1]) {
                // a chunk holds exactly kSweepChunk entries; padding reads the zero slot
                for (int32_t q = 0; q < kSweepChunk; ++q) {
                    const int64_t e = (int64_t)kSweepChunk * ch + q;
                    if (k < T.ptr[(size_t)row + 1]) {
                        const int32_t c = T.col[k], pc = posof[c];
                        int32_t slot;
                        if (pc >= p0)
                            slot = cur_base + (pc - p0);
                        else if (pc >= prev_p0 && pc < prev_p1)
                            slot = prev_base + (pc - prev_p0);
                        else
                            slot = 2 * kSweepPos + ext_slot[c];
                        eslot[e] = (uint16_t)slot;
                        eval[e] = (V)T.val[k];
                        ++k;
                    } else {
                        eslot[e] = (uint16_t)kSweepZeroSlot;
                        eval[e] = (V)0;
                    }
                }
                if (seg) crow[ch] = (uint16_t)((k == T.ptr[(size_t)row + 1] ? 0x8000 : 0) | (p - p0));
                ++ch;
            }
            if (hd) dg[p - p0] = (V)(1.0 / (*diag)[row]);  // the sweep multiplies by the reciprocal
        }
        while (lvl < l1) {
            ++lvl;
            lev_off[lvl - l0] = npos;
            lev_chunk[lvl - l0] = ch;
        }
        rchunk[npos] = (uint16_t)ch;
        // segmented scheme: bits 16..23 of a level's chunk offset hold its longest row in
        // chunks, which bounds the scan shifts the level needs
        if (seg)
            for (int32_t l = l0; l < l1; ++l) lev_chunk[l - l0] |= (int32_t)(std::min<int64_t>(maxchunks(l), 255) << 16);
        // the previous batch of the run learns this batch's size and older inputs,
        // so they are gathered while the previous batch is being solved
        if (bi > 0) {
            int32_t *ph = reinterpret_cast<int32_t *>(sw.blob.data() + sw.batch_off[(size_t)nbatches() - 1]);
            ph[8] = (int32_t)size;
            ph[9] = npos;
            ph[10] = (int32_t)next;
            int32_t *pnext = ph + kSweepHdr + 2 * (ph[0] + 1) + ph[1] + ph[3];  // next_ext of that blob
            for (int64_t j = 0; j < next; ++j) pnext[j] = ext[(size_t)j];
        }
        sw.batch_off.push_back((int64_t)sw.blob.size());
        batch_rows.push_back(npos);
        batch_nnz.push_back(nent);
        prev_p0 = p0;
        prev_p1 = p1;
    };

    auto close_batch = [&]() {
        if (bl0 >= 0) serialize(bl0, bl1);
        bl0 = -1;
    };
    auto close_run = [&]() {
        close_batch();
        if (run_b0 >= 0 && nbatches() > run_b0) {
            int64_t rows = 0, nnz = 0;
            for (int32_t bb = run_b0; bb < nbatches(); ++bb) {
                rows += batch_rows[(size_t)bb];
                nnz += batch_nnz[(size_t)bb];
            }
            sw.segs.push_back({-1, run_b0, nbatches(), rows, nnz, scheme});
        }
        run_b0 = -1;
        prev_p0 = prev_p1 = -1;
    };
    auto fits = [&](int64_t nlev, int64_t npos, int64_t nent, int64_t next, int64_t nchk) {
        (void)nent;
        return nlev <= kSweepLevels && npos <= kSweepPos && next <= kSweepExt &&
               blob_bytes(nlev, npos, next, nchk, hd, vb, seg) <= kSweepBlob;
    };
    for (int32_t l = 0; l < lv.nlev(); ++l) {
        const int64_t w = lv.ptr[(size_t)l + 1] - lv.ptr[l];
        const int64_t ne = entries(l), nc = chunks(l);
        if (w > kSweepRows || nc > kSweepLevEnt || (seg && maxchunks(l) > 64)) {
            close_run();
            sw.segs.push_back({l, -1, -1, w, ne, 0});
            continue;
        }
        if (bl0 >= 0) {
            // extend the open batch with level l if it still fits
            ++stamp;
            int64_t ext_now = 0;
            for (int32_t ll = bl0; ll <= l; ++ll) ext_now += new_ext(ll, lv.ptr[bl0]);
            if (fits(l - bl0 + 1, bpos + w, bent + ne, ext_now, bchk + nc)) {
                bl1 = l + 1;
                bpos += w;
                bent += ne;
                bchk += nc;
                continue;
            }
            close_batch();
        }
        // start a new batch with level l (the previous batch is now the last closed one)
        ++stamp;
        const int64_t e1 = new_ext(l, lv.ptr[l]);
        if (!fits(1, w, ne, e1, nc)) {
            close_run();
            sw.segs.push_back({l, -1, -1, w, ne, 0});
            continue;
        }
        if (run_b0 < 0) run_b0 = nbatches();
        bl0 = l;
        bl1 = l + 1;
        bpos = w;
        bent = ne;
        bchk = nc;
    }
    close_run();
    return sw;
}

int32_t lanes_for(double avg)
{
    int32_t g = 2;
    while (g < 64 && g < avg) g *= 2;
    return g;
}

// Lanes per row of a CSR product and entries per lane loaded at once: two rows
// per lane group with 4 lanes up to 8 entries per row on average, 8 lanes up to
// 16 (2 entries per lane) and up to 32 (4), 16 lanes up to 64 and 32 lanes up to
// 128 (3 entries per lane: fewer registers than 4, more wavefronts in flight; 3-5%
// faster on the products with Y~ and Y~^T, measured alternating as in the S~ steps);
// one row per 64-lane group beyond.
int32_t spmv_lanes(double avg)
{
    if (avg <= 8.0) return 4;
    if (avg <= 32.0) return 8;
    if (avg <= 64.0) return 16;
    if (avg <= 128.0) return 32;
    return 64;
}

int32_t spmv_unroll(double avg) { return avg <= 16.0 ? 2 : (avg <= 32.0 ? 4 : 3); }

SpmvPlan plan_spmv(const Csr &a)
{
    SpmvPlan pl;
    double avg = a.nrows ? (double)a.nnz() / (double)a.nrows : 1.0;
    pl.lanes = a.nnz() > 0 ? spmv_lanes(avg) : 2;  // the paired-row kernel needs an entry to clamp to
    pl.unroll = spmv_unroll(avg);
    pl.long_thresh = std::max<int32_t>(32 * pl.lanes, 2048);
    const int32_t seg = 4096;
    pl.seg_ptr.push_back(0);
    for (int32_t i = 0; i < a.nrows; ++i) {
        int32_t b = a.ptr[i], e = a.ptr[(size_t)i + 1];
        if (e - b <= pl.long_thresh) continue;
        pl.long_rows.push_back(i);
        for (int32_t s = b; s < e; s += seg) {
            pl.seg_beg.push_back(s);
            pl.seg_end.push_back(std::min(s + seg, e));
        }
        pl.seg_ptr.push_back((int32_t)pl.seg_beg.size());
    }
    return pl;
}

// ---------------------------------------------------------------- ILUP

struct Cand {
    double mag;
    double v;
    int32_t key;
};

// Entries kept by the dropping rule of Algorithm 4: v != 0 and |v| >= tau,
// then the p largest |v| (ties to the smaller key). Order of the result is
// unspecified.
void keep_largest(std::vector<Cand> &c, int64_t p, double tau)
{
    auto last = std::remove_if(c.begin(), c.end(), [tau](const Cand &e) { return !(e.v != 0.0 && e.mag >= tau); });
    c.erase(last, c.end());
    if ((int64_t)c.size() > p) {
        auto before = [](const Cand &x, const Cand &y) {
            return x.mag > y.mag || (x.mag == y.mag && x.key < y.key);
        };
        std::nth_element(c.begin(), c.begin() + p, c.end(), before);
        c.resize((size_t)p);
    }
}

double modified_pivot(int64_t j1, int64_t n, double colmax, double small)
{
    // Algorithm 6: beta = 10^(-2(1 - j/n)), value max(beta ||A(:,j)||_inf, small)
    double beta = std::pow(10.0, -2.0 * (1.0 - (double)j1 / (double)n));
    double v = beta * colmax;
    return v > small ? v : small;
}

}  // namespace

// Section 3.2: Y~ = L2 L1^{-1} computed once and stored as a sparse matrix. Row i
// of Y~ is the y with y L1 = l, l = row i of L2, i.e. the back substitution
// L1^T y^T = l^T with a sparse right-hand side: y_j = l_j - sum_{k>j} y_k L1(k,j).
// The positions are finalised from the highest down (a max-priority queue holds
// the positions reached so far; a position enters it once, from l's pattern or
// from the first kept y_k whose row of L1 has an entry in its column), so each
// y_j is complete when it leaves the queue. A finished y_k that is zero or below
// ytau in magnitude is dropped before it reaches any lower position, as the ILUP
// drops entries of L; a kept one is pushed down: y_j = y_j - (y_k * L1(k,j)),
// separately rounded, in the order the y_k finish. Rows are independent, so
// blocks of rows run on host threads and are concatenated in row order.
void build_explicit_Y(Ctx &c)
{
    const Csr &L1 = c.L1, &L2 = c.L2;
    const int32_t n = (int32_t)c.n, k = L2.nrows;
    const double ytau = c.prm.ytau;
    struct Part {
        std::vector<int32_t> len, col;
        std::vector<double> val;
    };
    const int32_t nthreads =
        (int32_t)std::max<int64_t>(1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 16,
                                                         ((int64_t)k + 1023) / 1024}));
    std::vector<Part> parts((size_t)nthreads);
    auto work = [&](int32_t t) {
        const int32_t r0 = (int32_t)((int64_t)k * t / nthreads), r1 = (int32_t)((int64_t)k * (t + 1) / nthreads);
        Part &out = parts[(size_t)t];
        std::vector<double> x((size_t)n, 0.0);
        std::vector<int32_t> stamp((size_t)n, -1);  // row index that queued the position
        std::priority_queue<int32_t> queue;
        std::vector<std::pair<int32_t, double>> row;
        for (int32_t i = r0; i < r1; ++i) {
            for (int32_t e = L2.ptr[i]; e < L2.ptr[(size_t)i + 1]; ++e) {
                x[(size_t)L2.col[e]] = L2.val[e];
                stamp[(size_t)L2.col[e]] = i;
                queue.push(L2.col[e]);
            }
            row.clear();
            while (!queue.empty()) {
                const int32_t kk = queue.top();
                queue.pop();
                const double yk = x[(size_t)kk];
                if (yk == 0.0 || std::fabs(yk) < ytau) continue;
                row.emplace_back(kk, yk);
                for (int32_t e = L1.ptr[kk]; e < L1.ptr[(size_t)kk + 1]; ++e) {
                    const int32_t j = L1.col[e];
                    if (stamp[(size_t)j] != i) {
                        stamp[(size_t)j] = i;
                        x[(size_t)j] = 0.0;
                        queue.push(j);
                    }
                    const double prod = yk * L1.val[e];
                    x[(size_t)j] = x[(size_t)j] - prod;
                }
            }
            out.len.push_back((int32_t)row.size());
            for (auto it = row.rbegin(); it != row.rend(); ++it) {
                out.col.push_back(it->first);
                out.val.push_back(it->second);
            }
        }
    };
    if (nthreads == 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        for (int32_t t = 0; t < nthreads; ++t) pool.emplace_back(work, t);
        for (std::thread &th : pool) th.join();
    }
    Csr &Y = c.Y;
    Y = Csr{};
    Y.nrows = k;
    Y.ncols = n;
    Y.ptr.assign((size_t)k + 1, 0);
    int64_t total = 0;
    for (const Part &pt : parts) total += (int64_t)pt.col.size();
    if (total > kMaxIdx) throw std::bad_alloc();
    Y.col.reserve((size_t)total);
    Y.val.reserve((size_t)total);
    int32_t i = 0;
    for (const Part &pt : parts) {
        for (int32_t len : pt.len) {
            Y.ptr[(size_t)i + 1] = Y.ptr[(size_t)i] + len;
            ++i;
        }
        Y.col.insert(Y.col.end(), pt.col.begin(), pt.col.end());
        Y.val.insert(Y.val.end(), pt.val.begin(), pt.val.end());
    }
    c.YT = transpose(Y);
    // The device copy takes Y~'s rows in the order of their first column (rows without
    // entries last, ties by row), so that rows near each other in the launch gather nearby
    // entries of their input, and the columns of its transpose follow that order: the
    // (m-n)-vectors of the S~ steps live in this order on the device. The products'
    // row sums are unchanged; only the order of the entries of those vectors differs.
    std::vector<int32_t> order((size_t)k);
    for (int32_t r = 0; r < k; ++r) order[(size_t)r] = r;
    auto first_col = [&](int32_t r) { return Y.ptr[(size_t)r + 1] > Y.ptr[r] ? Y.col[Y.ptr[r]] : n; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return first_col(a) < first_col(b); });
    c.yperm = order;
    c.yperm_inv.assign((size_t)k, 0);
    for (int32_t r = 0; r < k; ++r) c.yperm_inv[(size_t)order[(size_t)r]] = r;
    Csr &D = c.Yd;
    D = Csr{};
    D.nrows = k;
    D.ncols = n;
    D.ptr.assign((size_t)k + 1, 0);
    D.col.reserve(Y.col.size());
    D.val.reserve(Y.val.size());
    for (int32_t r = 0; r < k; ++r) {
        const int32_t src = order[(size_t)r];
        D.col.insert(D.col.end(), Y.col.begin() + Y.ptr[src], Y.col.begin() + Y.ptr[(size_t)src + 1]);
        D.val.insert(D.val.end(), Y.val.begin() + Y.ptr[src], Y.val.begin() + Y.ptr[(size_t)src + 1]);
        D.ptr[(size_t)r + 1] = (int32_t)D.col.size();
    }
    c.YdT = transpose(D);
    c.plY = plan_spmv(c.Yd);
    c.plYT = plan_spmv(c.YdT);
    // diag(S~) = 1 + (Y~ Y~^T)_ii for the Jacobi-preconditioned CG steps, in device order
    c.cg_diag.clear();
    if (c.prm.cg_precond == RSILU_CG_JACOBI) {
        c.cg_diag.assign((size_t)k, 1.0);
        for (int32_t r = 0; r < k; ++r) {
            double s = 0.0;
            for (int32_t e = D.ptr[r]; e < D.ptr[(size_t)r + 1]; ++e) {
                const double sq = D.val[e] * D.val[e];
                s = s + sq;
            }
            c.cg_diag[(size_t)r] = 1.0 + s;
        }
    }
}

// Section 3.2 lets an approximation S^ of S~ stand in for it when that is cheaper to
// solve with; RSILU_S_CHEB takes M_b^{-1} = the polynomial in S~ of K Chebyshev steps
// over [1, b]. S~ = I + Y~ Y~^T has its spectrum in [1, lambda_max]; b is 1.05 times a
// power-iteration estimate of lambda_max (50 products from the all-ones vector, the
// last Rayleigh quotient). K is the smallest even degree with (b - 1) / T_K(sigma) <=
// poly_delta, sigma = (b + 1)/(b - 1) (then 1 + (t - 1) r_K(t) stays within
// poly_delta of 1 on [1, b], and positive beyond b for even K), unless poly_degree
// fixes it. The step coefficients of the three-term recurrence are formed here once:
// theta = (b + 1)/2, delta = (b - 1)/2, rho_0 = delta/theta, rho_{j+1} = 1/(2 theta/delta
// - rho_j), c1_j = rho_{j+1} rho_j, c2_j = 2 rho_{j+1}/delta.
void build_chebyshev(Ctx &c)
{
    const int64_t k = c.L2.nrows, n = c.n;
    c.cheb_c1.clear();
    c.cheb_c2.clear();
    c.cheb_b = 1.0;
    c.cheb_K = 0;
    c.cheb_omega = 1.0;
    if (k == 0) return;
    // S~ d = d + Y~ (Y~^T d): explicit, or L2 L1^{-1} L1^{-T} L2^T d
    std::vector<double> g((size_t)n), t((size_t)n), q((size_t)k);
    auto spmv = [](const Csr &a, const double *x, double *y) {
        for (int32_t i = 0; i < a.nrows; ++i) {
            double sum = 0.0;
            for (int32_t e = a.ptr[i]; e < a.ptr[(size_t)i + 1]; ++e) sum += a.val[e] * x[a.col[e]];
            y[i] = sum;
        }
    };
    auto S = [&](const std::vector<double> &d, std::vector<double> &out) {
        if (yexplicit(c)) {
            spmv(c.YT, d.data(), g.data());
            spmv(c.Y, g.data(), q.data());
        } else {
            spmv(c.L2T, d.data(), g.data());
            for (int64_t r = n - 1; r >= 0; --r) {  // L1^T t = g (unit upper, by rows of L1^T)
                double sum = g[(size_t)r];
                for (int32_t e = c.L1T.ptr[r]; e < c.L1T.ptr[(size_t)r + 1]; ++e) sum -= c.L1T.val[e] * t[c.L1T.col[e]];
                t[(size_t)r] = sum;
            }
            for (int64_t r = 0; r < n; ++r) {  // L1 g = t
                double sum = t[(size_t)r];
                for (int32_t e = c.L1.ptr[r]; e < c.L1.ptr[(size_t)r + 1]; ++e) sum -= c.L1.val[e] * g[c.L1.col[e]];
                g[(size_t)r] = sum;
            }
            spmv(c.L2, g.data(), q.data());
        }
        for (int64_t i = 0; i < k; ++i) out[(size_t)i] = d[(size_t)i] + q[(size_t)i];
    };
    std::vector<double> v((size_t)k, 1.0 / std::sqrt((double)k)), w((size_t)k);
    double lam = 1.0;
    for (int it = 0; it < 50; ++it) {
        S(v, w);
        double vw = 0.0, ww = 0.0;
        for (int64_t i = 0; i < k; ++i) {
            vw += v[(size_t)i] * w[(size_t)i];
            ww += w[(size_t)i] * w[(size_t)i];
        }
        lam = vw;
        const double nw = std::sqrt(ww);
        if (!(nw > 0.0) || !std::isfinite(nw)) break;
        for (int64_t i = 0; i < k; ++i) v[(size_t)i] = w[(size_t)i] / nw;
    }
    if (!(lam > 1.0) || !std::isfinite(lam)) return;  // S~ = I: M_b^{-1} = I
    const double b = 1.05 * lam;
    const double sigma = (b + 1.0) / (b - 1.0);
    int32_t K = c.prm.poly_degree;
    if (K == 0) {
        K = 2;
        while (K < 512 && (b - 1.0) / std::cosh(K * std::acosh(sigma)) > c.prm.poly_delta) K += 2;
    }
    c.cheb_b = b;
    c.cheb_K = K;
    // a degree that misses the bound (b - 1) eps_K <= poly_delta: the input scaled by
    // 1 / (1 + eps_K) keeps M_b^{-1} positive definite
    const double epsK = 1.0 / std::cosh(K * std::acosh(sigma));
    c.cheb_omega = (b - 1.0) * epsK <= c.prm.poly_delta ? 1.0 : 1.0 / (1.0 + epsK);
    const double theta = (b + 1.0) / 2.0, half = (b - 1.0) / 2.0;
    const double sig = theta / half;
    double rho = 1.0 / sig;
    for (int32_t j = 0; j < K; ++j) {
        const double rho_new = 1.0 / (2.0 * sig - rho);
        c.cheb_c1.push_back(rho_new * rho);
        c.cheb_c2.push_back(2.0 * rho_new / half);
        rho = rho_new;
    }
    c.cheb_theta = theta;
}

// S~ = I + Y~ Y~^T with Y~^T = L1^{-T} L2^T, factored by Cholesky (Section 3.2),
// packed lower factor by rows.
rsilu_status_t build_dense_S(Ctx &c)
{
    const int64_t n = c.n;
    const int64_t k = c.L2.nrows;  // rows of A2 (m - n, less the removed rows of A1)
    if (k > 16384 || k * n > (int64_t)1 << 28) return RSILU_EINVAL;
    // Y^T = L1^{-T} L2^T, one column (row of Y) per row of L2
    std::vector<double> Y((size_t)(k * n), 0.0);  // row-major k x n
    for (int64_t i = 0; i < k; ++i) {
        double *y = &Y[(size_t)(i * n)];
        for (int32_t e = c.L2.ptr[i]; e < c.L2.ptr[(size_t)i + 1]; ++e) y[c.L2.col[e]] = c.L2.val[e];
        for (int64_t r = n - 1; r >= 0; --r) {  // L1^T y = l2_i, backward
            double s = y[r];
            for (int32_t e = c.L1T.ptr[r]; e < c.L1T.ptr[(size_t)r + 1]; ++e) s -= c.L1T.val[e] * y[c.L1T.col[e]];
            y[r] = s;
        }
    }
    // S~ = I + Y Y^T, lower Cholesky factor, packed by rows
    c.sfac.assign((size_t)(k * (k + 1) / 2), 0.0);
    auto at = [](int64_t i, int64_t jj) { return (size_t)(i * (i + 1) / 2 + jj); };
    for (int64_t i = 0; i < k; ++i) {
        const double *yi = &Y[(size_t)(i * n)];
        for (int64_t jj = 0; jj <= i; ++jj) {
            const double *yj = &Y[(size_t)(jj * n)];
            double s = (i == jj) ? 1.0 : 0.0;
            for (int64_t t = 0; t < n; ++t) s += yi[t] * yj[t];
            c.sfac[at(i, jj)] = s;
        }
    }
    for (int64_t jj = 0; jj < k; ++jj) {
        double d = c.sfac[at(jj, jj)];
        for (int64_t t = 0; t < jj; ++t) d -= c.sfac[at(jj, t)] * c.sfac[at(jj, t)];
        if (!(d > 0.0) || !std::isfinite(d)) return RSILU_BREAKDOWN;
        d = std::sqrt(d);
        c.sfac[at(jj, jj)] = d;
        for (int64_t i = jj + 1; i < k; ++i) {
            double s = c.sfac[at(i, jj)];
            for (int64_t t = 0; t < jj; ++t) s -= c.sfac[at(i, t)] * c.sfac[at(jj, t)];
            c.sfac[at(i, jj)] = s / d;
        }
    }
    return RSILU_OK;
}

rsilu_status_t build_factorization(Ctx &c, int64_t m, int64_t n, const int64_t *rowptr,
                                   const int32_t *colind, const double *val)
{
    const rsilu_params_t &P = c.prm;
    if (n < 1 || m < n || m > kMaxIdx || !rowptr || (rowptr[m] > 0 && (!colind || !val)))
        return RSILU_EINVAL;
    if (P.p < 0 || !(P.tau >= 0.0) || !(P.mu > 0.0 && P.mu <= 1.0) || !(P.small > 0.0) ||
        !std::isfinite(P.tau) || P.maxit < 0 || P.poll < 1 ||
        (P.smode != RSILU_S_AUTO && P.smode != RSILU_S_IDENTITY && P.smode != RSILU_S_DENSE &&
         P.smode != RSILU_S_NONE && P.smode != RSILU_S_CG && P.smode != RSILU_S_CHEB) ||
        (P.krylov != RSILU_KRYLOV_PCGLS && P.krylov != RSILU_KRYLOV_LSQR) || (P.graph != 0 && P.graph != 1) ||
        P.sweep < RSILU_SWEEP_AUTO || P.sweep > RSILU_SWEEP_ROWS ||
        (P.krylov == RSILU_KRYLOV_LSQR &&
         (P.form != RSILU_FORM_ALG2 || P.trsv == RSILU_TRSV_SYNCFREE ||
          (P.smode != RSILU_S_AUTO && P.smode != RSILU_S_NONE && P.smode != RSILU_S_DENSE &&
           P.smode != RSILU_S_CHEB))) ||
        (P.smode == RSILU_S_CHEB &&
         (P.trsv == RSILU_TRSV_SYNCFREE || P.poly_degree < 0 || P.poly_degree > 512 || !(P.poly_delta > 0.0) ||
          !(P.poly_delta < 1.0) || (P.precision == RSILU_PREC_FP32 && P.ystore != RSILU_Y_EXPLICIT))) ||
        (P.smode == RSILU_S_CG &&
         (P.precision != RSILU_PREC_FP64 || P.trsv == RSILU_TRSV_SYNCFREE || P.cg_steps < 1 || P.cg_steps > 256)) ||
        (P.cg_precond != RSILU_CG_NONE && P.cg_precond != RSILU_CG_JACOBI) ||
        (P.cg_precond == RSILU_CG_JACOBI && (P.smode != RSILU_S_CG || P.ystore != RSILU_Y_EXPLICIT)) ||
        (P.ystore != RSILU_Y_IMPLICIT && P.ystore != RSILU_Y_EXPLICIT) || !(P.ytau >= 0.0) || !std::isfinite(P.ytau) ||
        (P.ystore == RSILU_Y_EXPLICIT && (P.smode == RSILU_S_DENSE || P.trsv == RSILU_TRSV_SYNCFREE)) ||
        (P.form != RSILU_FORM_ALG3 && P.form != RSILU_FORM_ALG2) ||
        (P.precision != RSILU_PREC_FP64 && P.precision != RSILU_PREC_FP32) ||
        (P.precision == RSILU_PREC_FP32 && (P.trsv == RSILU_TRSV_SYNCFREE || P.smode == RSILU_S_DENSE)) ||
        (P.smode != RSILU_S_AUTO && (P.smode < RSILU_S_IDENTITY || P.smode > RSILU_S_CHEB)) ||
        (P.trsv != RSILU_TRSV_SYNCFREE && P.trsv != RSILU_TRSV_LEVELS && P.trsv != RSILU_TRSV_HYBRID))
        return RSILU_EINVAL;
    if (rowptr[0] != 0 || rowptr[m] > kMaxIdx) return RSILU_EINVAL;

    // ---- validate, strip explicit zeros (problem (1.1): A real, sparse, m >= n)
    Csr &A = c.A;
    A.nrows = (int32_t)m;
    A.ncols = (int32_t)n;
    A.ptr.assign((size_t)m + 1, 0);
    for (int64_t i = 0; i < m; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return RSILU_EINVAL;
        int32_t prev = -1;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            int32_t cc = colind[e];
            if (cc < 0 || cc >= n || cc <= prev || !std::isfinite(val[e])) return RSILU_EINVAL;
            prev = cc;
            if (val[e] != 0.0) {
                A.col.push_back(cc);
                A.val.push_back(val[e]);
            }
        }
        A.ptr[(size_t)i + 1] = (int32_t)A.col.size();
    }
    c.m = m;
    c.n = n;
    c.nnz_a = A.nnz();

    // ---- columns of A (rows ascending), Section 5.1 prescaling
    Csr AT = transpose(A);  // row j of AT = column j of A
    c.colnorm.assign((size_t)n, 1.0);
    std::vector<double> sval(AT.val.size());
    for (int32_t j = 0; j < (int32_t)n; ++j) {
        const int32_t b = AT.ptr[j], e = AT.ptr[(size_t)j + 1];
        double nrm = 1.0;
        if (P.colscale && e > b) {
            double s = 0.0;
            for (int32_t k = b; k < e; ++k) {
                double sq = AT.val[k] * AT.val[k];
                s = s + sq;
            }
            nrm = std::sqrt(s);
            if (nrm == 0.0) nrm = 1.0;
        }
        c.colnorm[j] = nrm;
        for (int32_t k = b; k < e; ++k) sval[k] = P.colscale ? AT.val[k] / nrm : AT.val[k];
    }

    // ---- Algorithm 4: left-looking ILUP over the columns
    const int64_t pcap = std::min<int64_t>(P.p, m);
    std::vector<int32_t> &perm = c.perm;
    perm.resize((size_t)m);
    std::vector<int32_t> pos((size_t)m);
    for (int32_t i = 0; i < (int32_t)m; ++i) perm[i] = pos[i] = i;
    std::vector<int32_t> rc((size_t)m, 0);
    for (int32_t i = 0; i < (int32_t)m; ++i) rc[i] = A.ptr[(size_t)i + 1] - A.ptr[i];

    std::vector<int32_t> lptr(1, 0), lrow;  // columns of L~ (original row ids)
    std::vector<double> lval;
    std::vector<std::vector<std::pair<int32_t, double>>> urows((size_t)n);  // U by rows (step)
    c.Udiag.assign((size_t)n, 0.0);

    std::vector<double> w((size_t)m, 0.0);
    std::vector<int32_t> stamp((size_t)m, -1);     // row touched in column j
    std::vector<int32_t> queued((size_t)n, -1);    // step queued in column j
    std::vector<int32_t> touched;
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> ready;
    std::vector<Cand> lc, uc;
    c.nmod = 0;

    for (int32_t j = 0; j < (int32_t)n; ++j) {
        touched.clear();
        double colmax = 0.0;
        for (int32_t k = AT.ptr[j]; k < AT.ptr[(size_t)j + 1]; ++k) {
            const int32_t i = AT.col[k];
            w[i] = sval[k];
            stamp[i] = j;
            touched.push_back(i);
            const double a = std::fabs(sval[k]);
            if (a > colmax) colmax = a;
            if (pos[i] < j && queued[pos[i]] != j) {
                queued[pos[i]] = j;
                ready.push(pos[i]);
            }
        }
        // Sparse triangular solve for U(1:j-1, j) and update of L(j:m, j):
        // steps are taken in increasing order; a step is final when popped
        // because only smaller steps update its row.
        uc.clear();
        while (!ready.empty()) {
            const int32_t k = ready.top();
            ready.pop();
            const double uk = w[perm[k]];
            if (uk == 0.0) continue;
            uc.push_back({std::fabs(uk), uk, k});
            for (int32_t e = lptr[k]; e < lptr[(size_t)k + 1]; ++e) {
                const int32_t r = lrow[e];
                const double prod = lval[e] * uk;
                w[r] = w[r] - prod;
                if (stamp[r] != j) {
                    stamp[r] = j;
                    touched.push_back(r);
                }
                const int32_t pr = pos[r];
                if (pr < j && queued[pr] != j) {
                    queued[pr] = j;
                    ready.push(pr);
                }
            }
        }
        // Candidates of the L column: unpivoted rows with a nonzero value.
        lc.clear();
        double amax = 0.0;
        for (int32_t r : touched) {
            if (pos[r] >= j && w[r] != 0.0) {
                const double a = std::fabs(w[r]);
                lc.push_back({a, w[r], r});
                if (a > amax) amax = a;
            }
        }
        // Algorithm 5 (pivot choice) and Algorithm 6 (modification).
        int32_t piv;
        double pv;
        if (lc.empty()) {
            piv = perm[j];
            pv = modified_pivot(j + 1, n, colmax, P.small);
            c.nmod++;
        } else {
            const double thr = P.mu * amax;
            const Cand *best = nullptr;
            for (const Cand &e : lc) {
                if (!(e.mag >= thr)) continue;
                if (!best) {
                    best = &e;
                    continue;
                }
                const int32_t re = rc[e.key], rb = rc[best->key];
                if (re != rb ? re < rb : (e.mag != best->mag ? e.mag > best->mag : e.key < best->key)) best = &e;
            }
            piv = best->key;
            pv = best->v;
            if (std::fabs(pv) < P.small) {
                pv = modified_pivot(j + 1, n, colmax, P.small);
                c.nmod++;
            }
        }
        // Interchange positions j and pos[piv].
        {
            const int32_t pp = pos[piv], rj = perm[j];
            perm[pp] = rj;
            pos[rj] = pp;
            perm[j] = piv;
            pos[piv] = j;
        }
        // Scale by the pivot, then drop (L after scaling, U on the exact values).
        size_t kept = 0;
        for (const Cand &e : lc) {
            if (e.key == piv) continue;
            const double l = e.v / pv;
            lc[kept++] = {std::fabs(l), l, e.key};
        }
        lc.resize(kept);
        keep_largest(lc, pcap, P.tau);
        keep_largest(uc, pcap, P.tau);
        if ((int64_t)lrow.size() + (int64_t)lc.size() > kMaxIdx) return RSILU_EINVAL;
        for (const Cand &e : lc) {
            lrow.push_back(e.key);
            lval.push_back(e.v);
        }
        lptr.push_back((int32_t)lrow.size());
        for (const Cand &e : uc) urows[e.key].push_back({j, e.v});
        c.Udiag[j] = pv;
        // rc(i) counts the entries of row i in the columns still to come.
        for (int32_t k = AT.ptr[j]; k < AT.ptr[(size_t)j + 1]; ++k) rc[AT.col[k]]--;
        for (int32_t r : touched) w[r] = 0.0;
    }

    // ---- the splitting (3.8): L1 (positions < n), L2 (positions >= n), U
    {
        std::vector<std::vector<std::pair<int32_t, double>>> r1((size_t)n), r2((size_t)(m - n));
        for (int32_t k = 0; k < (int32_t)n; ++k) {
            for (int32_t e = lptr[k]; e < lptr[(size_t)k + 1]; ++e) {
                const int32_t q = pos[lrow[e]];
                if (q < n)
                    r1[q].push_back({k, lval[e]});
                else
                    r2[(size_t)(q - n)].push_back({k, lval[e]});
            }
        }
        c.L1 = from_rows((int32_t)n, (int32_t)n, r1);
        c.L2 = from_rows((int32_t)(m - n), (int32_t)n, r2);
        c.U = from_rows((int32_t)n, (int32_t)n, urows);
    }
    c.L1T = transpose(c.L1);
    c.L2T = transpose(c.L2);
    c.UT = transpose(c.U);

    // ---- A_hat = P A D in pivot order, and its transpose
    {
        Csr &H = c.Ahat;
        H.nrows = (int32_t)m;
        H.ncols = (int32_t)n;
        H.ptr.assign((size_t)m + 1, 0);
        H.col.reserve(A.col.size());
        H.val.reserve(A.val.size());
        for (int32_t k = 0; k < (int32_t)m; ++k) {
            const int32_t i = perm[k];
            for (int32_t e = A.ptr[i]; e < A.ptr[(size_t)i + 1]; ++e) {
                H.col.push_back(A.col[e]);
                H.val.push_back(P.colscale ? A.val[e] / c.colnorm[A.col[e]] : A.val[e]);
            }
            H.ptr[(size_t)k + 1] = (int32_t)H.col.size();
        }
        c.AhatT = transpose(H);
    }

    // ---- level schedules
    c.lvL1 = kahn_levels(c.L1, c.L1T);
    c.lvL1T = kahn_levels(c.L1T, c.L1);
    c.lvU = kahn_levels(c.U, c.UT);
    c.lvUT = kahn_levels(c.UT, c.U);
    if ((int64_t)c.lvL1.rows.size() != n || (int64_t)c.lvU.rows.size() != n) return RSILU_EINVAL;

    // ---- schedules of the products and sync-free solves
    c.plA = plan_spmv(c.Ahat);
    c.plAT = plan_spmv(c.AhatT);
    c.plL2 = plan_spmv(c.L2);
    c.plL2T = plan_spmv(c.L2T);
    auto tri_lanes = [](const Csr &t) { return lanes_for(t.nrows ? (double)t.nnz() / t.nrows : 1.0); };
    c.chL1 = make_chunks(c.lvL1, 64 / tri_lanes(c.L1));
    c.chL1T = make_chunks(c.lvL1T, 64 / tri_lanes(c.L1T));
    c.chU = make_chunks(c.lvU, 64 / tri_lanes(c.U));
    const bool f32 = P.precision == RSILU_PREC_FP32;
    const int32_t sw = P.sweep;
    c.swL1 = f32 ? make_sweep<float>(c.L1, nullptr, c.lvL1, sw) : make_sweep<double>(c.L1, nullptr, c.lvL1, sw);
    c.swL1T = f32 ? make_sweep<float>(c.L1T, nullptr, c.lvL1T, sw) : make_sweep<double>(c.L1T, nullptr, c.lvL1T, sw);
    c.swU = f32 ? make_sweep<float>(c.U, &c.Udiag, c.lvU, sw) : make_sweep<double>(c.U, &c.Udiag, c.lvU, sw);
    // U^T (forward, Udiag on the diagonal) for Algorithm 2's M_a = (L1 U)^T (L1 U)
    c.chUT = make_chunks(c.lvUT, 64 / tri_lanes(c.UT));
    c.swUT = f32 ? make_sweep<float>(c.UT, &c.Udiag, c.lvUT, sw) : make_sweep<double>(c.UT, &c.Udiag, c.lvUT, sw);

    auto lo = [&](const Csr &T, const std::vector<double> *diag, const Levels &lv) {
        return f32 ? level_ordered<float>(T, diag, lv) : level_ordered<double>(T, diag, lv);
    };
    c.loL1 = lo(c.L1, nullptr, c.lvL1);
    c.loL1T = lo(c.L1T, nullptr, c.lvL1T);
    c.loU = lo(c.U, &c.Udiag, c.lvU);
    c.loUT = lo(c.UT, &c.Udiag, c.lvUT);

    // ---- S^ (Section 3.2)
    const bool yexp = P.ystore == RSILU_Y_EXPLICIT;
    c.smode = P.smode;
    if (c.smode == RSILU_S_AUTO)
        c.smode = (m - n > 0 && m - n <= 4096 && !f32 && !yexp)
                      ? RSILU_S_DENSE
                      : (P.krylov == RSILU_KRYLOV_LSQR ? RSILU_S_NONE : RSILU_S_IDENTITY);
    if (yexp) build_explicit_Y(c);
    if (c.smode == RSILU_S_DENSE && m > n) {
        const rsilu_status_t rc = build_dense_S(c);
        if (rc != RSILU_OK) return rc;
    } else if (c.smode != RSILU_S_NONE && c.smode != RSILU_S_CG && c.smode != RSILU_S_CHEB) {
        c.smode = RSILU_S_IDENTITY;
    }
    if (c.smode == RSILU_S_CHEB) build_chebyshev(c);
    return RSILU_OK;
}

// Section 3.4, adding rows: the factorization of A is kept (L1, U and the pivot
// order of A1). Each new row a, prescaled with the setup's column norms (a_hat =
// a D), joins A2 at the end of the row order, and its L2 row l solves
// U^T l^T = a_hat^T by forward substitution (products summed in entry order,
// separately rounded, then subtracted and divided by the diagonal); entries with
// |l_j| < tau, or zero, are dropped as in the ILUP's dropping of L. The products'
// plans, the transposes and, in dense mode, S~ are rebuilt. Every argument is
// checked before the handle changes.
rsilu_status_t append_rows(Ctx &c, int64_t count, const int64_t *rowptr, const int32_t *colind, const double *val)
{
    const int64_t n = c.n, m0 = c.m;
    if (count < 1 || !rowptr || rowptr[0] != 0 || m0 + count > kMaxIdx) return RSILU_EINVAL;
    if (rowptr[count] > 0 && (!colind || !val)) return RSILU_EINVAL;
    for (int64_t i = 0; i < count; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return RSILU_EINVAL;
        int32_t prev = -1;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t cc = colind[e];
            if (cc < 0 || cc >= n || cc <= prev || !std::isfinite(val[e])) return RSILU_EINVAL;
            prev = cc;
        }
    }
    if (c.A.nnz() + rowptr[count] > kMaxIdx) return RSILU_EINVAL;
    if (c.smode == RSILU_S_DENSE) {
        const int64_t k = (int64_t)c.L2.nrows + count;
        if (k > 16384 || k * n > (int64_t)1 << 28) return RSILU_EINVAL;
    }
    const bool scale = c.prm.colscale != 0;
    std::vector<double> y((size_t)n);
    for (int64_t i = 0; i < count; ++i) {
        std::fill(y.begin(), y.end(), 0.0);
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (val[e] == 0.0) continue;
            const int32_t cc = colind[e];
            const double ah = scale ? val[e] / c.colnorm[cc] : val[e];
            c.A.col.push_back(cc);
            c.A.val.push_back(val[e]);
            c.Ahat.col.push_back(cc);
            c.Ahat.val.push_back(ah);
            y[cc] = ah;
        }
        c.A.ptr.push_back((int32_t)c.A.col.size());
        c.A.nrows++;
        c.Ahat.ptr.push_back((int32_t)c.Ahat.col.size());
        c.Ahat.nrows++;
        // U^T l^T = a_hat^T: row j of U^T holds the entries U(i, j), i < j
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int32_t e = c.UT.ptr[j]; e < c.UT.ptr[(size_t)j + 1]; ++e) {
                const double prod = c.UT.val[e] * y[c.UT.col[e]];
                s = s + prod;
            }
            const double r = y[j] - s;
            y[j] = r / c.Udiag[j];
        }
        for (int64_t j = 0; j < n; ++j) {
            if (y[j] != 0.0 && std::fabs(y[j]) >= c.prm.tau) {
                c.L2.col.push_back((int32_t)j);
                c.L2.val.push_back(y[j]);
            }
        }
        c.L2.ptr.push_back((int32_t)c.L2.col.size());
        c.L2.nrows++;
        c.perm.push_back((int32_t)(m0 + i));
    }
    c.m = m0 + count;
    c.nnz_a = c.A.nnz();
    c.AhatT = transpose(c.Ahat);
    c.L2T = transpose(c.L2);
    c.plA = plan_spmv(c.Ahat);
    c.plAT = plan_spmv(c.AhatT);
    c.plL2 = plan_spmv(c.L2);
    c.plL2T = plan_spmv(c.L2T);
    if (c.smode == RSILU_S_DENSE) {
        const rsilu_status_t rc = build_dense_S(c);
        if (rc != RSILU_OK) return rc;
    }
    if (yexplicit(c)) build_explicit_Y(c);
    if (c.smode == RSILU_S_CHEB) build_chebyshev(c);
    // with removed A1 rows, W depends on the operator the new rows changed
    if (c.R.nrows > 0) return build_woodbury(c);
    return RSILU_OK;
}

namespace {

// x = T^{-1} b for a strictly triangular CSR T with an optional diagonal, rows
// ascending (lower) or descending (upper); products summed in entry order.
void host_trsv(const Csr &T, const double *diag, bool lower, const double *b, double *x)
{
    const int32_t n = T.nrows;
    for (int32_t q = 0; q < n; ++q) {
        const int32_t i = lower ? q : n - 1 - q;
        double s = 0.0;
        for (int32_t e = T.ptr[i]; e < T.ptr[(size_t)i + 1]; ++e) {
            const double prod = T.val[e] * x[T.col[e]];
            s = s + prod;
        }
        const double r = b[i] - s;
        x[i] = diag ? r / diag[i] : r;
    }
}

void host_spmv(const Csr &A, const double *x, double *y)
{
    for (int32_t i = 0; i < A.nrows; ++i) {
        double s = 0.0;
        for (int32_t e = A.ptr[i]; e < A.ptr[(size_t)i + 1]; ++e) s += A.val[e] * x[A.col[e]];
        y[i] = s;
    }
}

// w = (F F^T)^{-1} w for F packed lower by rows (k x k)
void host_chol_solve(const std::vector<double> &F, int64_t k, double *w)
{
    auto at = [](int64_t i, int64_t j) { return (size_t)(i * (i + 1) / 2 + j); };
    for (int64_t i = 0; i < k; ++i) {
        double s = w[i];
        for (int64_t j = 0; j < i; ++j) s -= F[at(i, j)] * w[j];
        w[i] = s / F[at(i, i)];
    }
    for (int64_t i = k - 1; i >= 0; --i) {
        double s = w[i];
        for (int64_t j = i + 1; j < k; ++j) s -= F[at(j, i)] * w[j];
        w[i] = s / F[at(i, i)];
    }
}

// h = M^{-1} z of Algorithm 2 (k = n) with the dense S~ (or none when m = n), in the
// factored form of the device path: g = L1^{-T} U^{-T} z, u = S~^{-1} L2 L1^{-1} g,
// h = U^{-1} L1^{-1} (g - L1^{-T} L2^T u).
void host_apply_alg2(const Ctx &c, const double *z, double *h)
{
    const int32_t n = (int32_t)c.n;
    const int64_t k = c.L2.nrows;
    std::vector<double> t((size_t)n), g((size_t)n), v((size_t)n);
    host_trsv(c.UT, c.Udiag.data(), true, z, t.data());
    host_trsv(c.L1T, nullptr, false, t.data(), g.data());
    if (k > 0 && !c.sfac.empty()) {
        host_trsv(c.L1, nullptr, true, g.data(), v.data());
        std::vector<double> u((size_t)k), gq((size_t)n), c2((size_t)n);
        host_spmv(c.L2, v.data(), u.data());
        host_chol_solve(c.sfac, k, u.data());
        host_spmv(c.L2T, u.data(), gq.data());
        host_trsv(c.L1T, nullptr, false, gq.data(), c2.data());
        for (int32_t i = 0; i < n; ++i) g[i] = g[i] - c2[i];
    }
    host_trsv(c.L1, nullptr, true, g.data(), v.data());
    host_trsv(c.U, c.Udiag.data(), false, v.data(), h);
}

Csr rows_of(const Csr &A, const std::vector<int32_t> &keep)
{
    Csr o;
    o.nrows = (int32_t)keep.size();
    o.ncols = A.ncols;
    o.ptr.assign(1, 0);
    for (int32_t i : keep) {
        for (int32_t e = A.ptr[i]; e < A.ptr[(size_t)i + 1]; ++e) {
            o.col.push_back(A.col[e]);
            o.val.push_back(A.val[e]);
        }
        o.ptr.push_back((int32_t)o.col.size());
    }
    return o;
}

}  // namespace

// W = I - R M^{-1} R^T for the removed A1 rows R, with the current Algorithm 2
// operator M^{-1} (host, FP64), and its packed lower Cholesky factor; also R^T
// and the products' plans. BREAKDOWN if W is not positive definite.
rsilu_status_t build_woodbury(Ctx &c)
{
    const int64_t n = c.n;
    const int64_t r = c.R.nrows;
    c.RT = transpose(c.R);
    c.plR = plan_spmv(c.R);
    c.plRT = plan_spmv(c.RT);
    c.wfac.assign((size_t)(r * (r + 1) / 2), 0.0);
    auto at = [](int64_t i, int64_t j) { return (size_t)(i * (i + 1) / 2 + j); };
    {
        std::vector<double> e((size_t)n), h((size_t)n), col((size_t)r);
        std::vector<double> Wd((size_t)(r * r));
        for (int64_t i = 0; i < r; ++i) {
            std::fill(e.begin(), e.end(), 0.0);
            for (int32_t q = c.R.ptr[i]; q < c.R.ptr[(size_t)i + 1]; ++q) e[c.R.col[q]] = c.R.val[q];
            host_apply_alg2(c, e.data(), h.data());
            host_spmv(c.R, h.data(), col.data());
            for (int64_t j = 0; j < r; ++j) Wd[(size_t)(j * r + i)] = (i == j ? 1.0 : 0.0) - col[j];
        }
        for (int64_t i = 0; i < r; ++i)
            for (int64_t j = 0; j <= i; ++j)
                c.wfac[at(i, j)] = 0.5 * (Wd[(size_t)(i * r + j)] + Wd[(size_t)(j * r + i)]);
    }
    for (int64_t j = 0; j < r; ++j) {
        double d = c.wfac[at(j, j)];
        for (int64_t t = 0; t < j; ++t) d -= c.wfac[at(j, t)] * c.wfac[at(j, t)];
        if (!(d > 0.0) || !std::isfinite(d)) return RSILU_BREAKDOWN;
        d = std::sqrt(d);
        c.wfac[at(j, j)] = d;
        for (int64_t i = j + 1; i < r; ++i) {
            double sum = c.wfac[at(i, j)];
            for (int64_t t = 0; t < j; ++t) sum -= c.wfac[at(i, t)] * c.wfac[at(j, t)];
            c.wfac[at(i, j)] = sum / d;
        }
    }
    return RSILU_OK;
}

// Section 3.4, removing rows (original indices, renumbered afterwards in their
// order): the factorization is kept. Removed rows of A2 leave L2 and S~ is
// refactored; removed rows of A1 leave A_hat and join R, and the preconditioner
// becomes M^{-1} + M^{-1} R^T W^{-1} R M^{-1}, W = I - R M^{-1} R^T, for every A1 row
// removed so far (C1 = C - R^T R, Woodbury). Needs Algorithm 2, FP64 and the dense
// S~ (the mode in which M approximates A^T A, not only its A1 part).
rsilu_status_t remove_rows(Ctx &c, int64_t count, const int64_t *rows)
{
    const int64_t m = c.m, n = c.n;
    if (c.prm.form != RSILU_FORM_ALG2 || c.prm.precision != RSILU_PREC_FP64 || c.smode != RSILU_S_DENSE ||
        c.prm.trsv == RSILU_TRSV_SYNCFREE)
        return RSILU_EINVAL;
    if (count < 1 || !rows || m - count < n) return RSILU_EINVAL;
    std::vector<int32_t> pos((size_t)m);
    for (int64_t p = 0; p < m; ++p) pos[c.perm[p]] = (int32_t)p;
    std::vector<char> gone_row((size_t)m, 0), gone_pos((size_t)m, 0);
    for (int64_t i = 0; i < count; ++i) {
        if (rows[i] < 0 || rows[i] >= m || gone_row[rows[i]]) return RSILU_EINVAL;
        gone_row[rows[i]] = 1;
        gone_pos[pos[rows[i]]] = 1;
    }
    const int64_t r_old = c.R.nrows;
    int64_t r_new = r_old;
    for (int64_t p = 0; p < n; ++p) r_new += gone_pos[p];
    if (r_new > 4096) return RSILU_EINVAL;
    // new numbering of the kept original rows
    std::vector<int32_t> renum((size_t)m, -1);
    std::vector<int32_t> kept_rows;
    for (int64_t i = 0; i < m; ++i)
        if (!gone_row[i]) {
            renum[i] = (int32_t)kept_rows.size();
            kept_rows.push_back((int32_t)i);
        }
    std::vector<int32_t> kept_pos, kept_l2, a1_gone;
    for (int64_t p = 0; p < m; ++p) {
        if (!gone_pos[p]) kept_pos.push_back((int32_t)p);
        else if (p < n) a1_gone.push_back((int32_t)p);
        if (p >= n && !gone_pos[p]) kept_l2.push_back((int32_t)(p - n));
    }
    // R grows by the removed A1 rows of A_hat (in position order)
    {
        Csr add = rows_of(c.Ahat, a1_gone);
        if (c.R.nrows == 0) {
            c.R = add;
        } else {
            for (int32_t i = 0; i < add.nrows; ++i) {
                for (int32_t e = add.ptr[i]; e < add.ptr[(size_t)i + 1]; ++e) {
                    c.R.col.push_back(add.col[e]);
                    c.R.val.push_back(add.val[e]);
                }
                c.R.ptr.push_back((int32_t)c.R.col.size());
                c.R.nrows++;
            }
        }
    }
    std::vector<int32_t> perm;
    for (int32_t p : kept_pos) perm.push_back(renum[c.perm[p]]);
    c.perm = perm;
    c.A = rows_of(c.A, kept_rows);
    c.Ahat = rows_of(c.Ahat, kept_pos);
    c.L2 = rows_of(c.L2, kept_l2);
    c.m = m - count;
    c.nnz_a = c.A.nnz();
    c.AhatT = transpose(c.Ahat);
    c.L2T = transpose(c.L2);
    c.plA = plan_spmv(c.Ahat);
    c.plAT = plan_spmv(c.AhatT);
    c.plL2 = plan_spmv(c.L2);
    c.plL2T = plan_spmv(c.L2T);
    c.sfac.clear();
    if (c.L2.nrows > 0) {
        const rsilu_status_t rc = build_dense_S(c);
        if (rc != RSILU_OK) return rc;
    }
    return c.R.nrows > 0 ? build_woodbury(c) : RSILU_OK;
}

// ---------------------------------------------------------------- device layout

namespace {
struct Bump {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        size_t o = off;
        off += std::max<size_t>(bytes, 8);
        return o;
    }
};

DevCsrOff place_csr(Bump &b, const Csr &a, int32_t vbytes = 8)
{
    DevCsrOff o;
    o.nrows = a.nrows;
    o.ncols = a.ncols;
    o.nnz = a.nnz();
    o.vbytes = vbytes;
    o.ptr = b.take(sizeof(int32_t) * a.ptr.size());
    o.col = b.take(sizeof(int32_t) * a.col.size());
    o.val = b.take((size_t)vbytes * a.val.size());
    return o;
}

DevPlanOff place_plan(Bump &b, const SpmvPlan &pl)
{
    DevPlanOff o;
    o.nlong = (int32_t)pl.long_rows.size();
    o.nseg = (int32_t)pl.seg_beg.size();
    o.lanes = pl.lanes;
    o.unroll = pl.unroll;
    o.long_thresh = pl.long_thresh;
    o.long_rows = b.take(sizeof(int32_t) * pl.long_rows.size());
    o.seg_ptr = b.take(sizeof(int32_t) * pl.seg_ptr.size());
    o.seg_beg = b.take(sizeof(int32_t) * pl.seg_beg.size());
    o.seg_end = b.take(sizeof(int32_t) * pl.seg_end.size());
    return o;
}

DevTriOff place_tri(Bump &b, const Csr &a, bool diag, const Levels &lv, const Chunks &ch, const Sweep &sw,
                    const LoTri &lo, size_t n, int32_t vbytes)
{
    DevTriOff o;
    o.lev = b.take(sizeof(int32_t) * lv.ptr.size());
    o.lo = place_csr(b, lo.a, vbytes);
    o.ldiag = diag ? b.take((size_t)vbytes * n) : 0;
    o.lrec = b.take(lo.rec.size());
    o.blob = b.take(sw.blob.size());
    o.a = place_csr(b, a, vbytes);
    o.diag = diag ? b.take((size_t)vbytes * n) : 0;
    o.rows = b.take(sizeof(int32_t) * lv.rows.size());
    o.chunk = b.take(sizeof(int32_t) * ch.ptr.size());
    o.nchunks = (int32_t)ch.ptr.size() - 1;
    o.cap = ch.cap;
    o.lanes = 64 / ch.cap;
    o.nlev = lv.nlev();
    return o;
}
}  // namespace

void plan_layout(Ctx &c)
{
    Bump b;
    Layout &L = c.lay;
    const size_t m = (size_t)c.m, n = (size_t)c.n, k = (size_t)c.L2.nrows;
    L.state = b.take(4096);
    L.A = place_csr(b, c.Ahat);
    L.AT = place_csr(b, c.AhatT);
    const int32_t vb = fp32(c) ? 4 : 8;  // factor values
    L.L2 = place_csr(b, c.L2, vb);
    L.L2T = place_csr(b, c.L2T, vb);
    L.pA = place_plan(b, c.plA);
    L.pAT = place_plan(b, c.plAT);
    L.pL2 = place_plan(b, c.plL2);
    L.pL2T = place_plan(b, c.plL2T);
    if (yexplicit(c)) {
        L.Y = place_csr(b, c.Yd, vb);
        L.YT = place_csr(b, c.YdT, vb);
        L.pY = place_plan(b, c.plY);
        L.pYT = place_plan(b, c.plYT);
        L.yperm = b.take(sizeof(int32_t) * std::max<size_t>(k, 1));
        L.yperm_inv = b.take(sizeof(int32_t) * std::max<size_t>(k, 1));
        L.yk = b.take(sizeof(double) * std::max<size_t>(k, 1));
    }
    L.L1f = place_tri(b, c.L1, false, c.lvL1, c.chL1, c.swL1, c.loL1, n, vb);
    L.L1b = place_tri(b, c.L1T, false, c.lvL1T, c.chL1T, c.swL1T, c.loL1T, n, vb);
    L.Ub = place_tri(b, c.U, true, c.lvU, c.chU, c.swU, c.loU, n, vb);
    L.UTf = place_tri(b, c.UT, true, c.lvUT, c.chUT, c.swUT, c.loUT, n, vb);
    L.perm = b.take(sizeof(int32_t) * m);
    L.colnorm = b.take(sizeof(double) * n);
    L.sfac = b.take(sizeof(double) * c.sfac.size());
    if (c.R.nrows > 0) {
        L.R = place_csr(b, c.R);
        L.RT = place_csr(b, c.RT);
        L.pR = place_plan(b, c.plR);
        L.pRT = place_plan(b, c.plRT);
        L.wfac = b.take(sizeof(double) * c.wfac.size());
        L.wr = b.take(sizeof(double) * (size_t)c.R.nrows);
        L.wz = b.take(sizeof(double) * n);
        L.wh = b.take(sizeof(double) * n);
    }
    for (size_t *o : {&L.xh, &L.p, &L.z, &L.h, &L.t, &L.y, &L.v, &L.g, &L.gp, &L.s2, &L.c2})
        *o = b.take(sizeof(double) * n);
    L.r = b.take(sizeof(double) * m);
    L.q = b.take(sizeof(double) * m);
    L.u = b.take(sizeof(double) * std::max<size_t>(k, 1));
    L.lo_rhs = b.take(sizeof(double) * n);
    L.lo_add = b.take(sizeof(double) * n);
    if (fp32(c)) {
        L.f32a = b.take(sizeof(float) * m);
        L.f32b = b.take(sizeof(float) * m);
    }
    if (c.smode == RSILU_S_CG || c.smode == RSILU_S_CHEB)
        for (size_t *o : {&L.cg_w, &L.cg_r, &L.cg_p, &L.cg_q}) *o = b.take(sizeof(double) * std::max<size_t>(k, 1));
    if (c.smode == RSILU_S_CHEB) L.cheb = b.take(sizeof(double) * std::max<size_t>(2 * (size_t)c.cheb_K, 1));
    if (c.smode == RSILU_S_CG) L.cg_part = b.take(sizeof(double) * 3 * (size_t)kCgParts);
    if (c.smode == RSILU_S_CG && !c.cg_diag.empty()) {
        L.cg_d = b.take(sizeof(double) * std::max<size_t>(k, 1));
        L.cg_z = b.take(sizeof(double) * std::max<size_t>(k, 1));
    }
    if (c.prm.krylov == RSILU_KRYLOV_LSQR)
        for (size_t *o : {&L.l_v, &L.l_mv, &L.l_w}) *o = b.take(sizeof(double) * n);
    // one partial per block of the largest reduction (a product's blocks hold
    // kBlock / lanes rows; dot products use at most 2048 blocks), plus one per long row
    auto blocks = [](int64_t rows, int32_t lanes) {
        const int64_t per = 256 / std::max<int32_t>(lanes, 1);
        return (rows + per - 1) / per;
    };
    const int64_t nparts = std::max<int64_t>({(int64_t)2048, blocks(c.Ahat.nrows, c.plA.lanes),
                                              blocks(c.AhatT.nrows, c.plAT.lanes), blocks(c.L2.nrows, c.plL2.lanes),
                                              blocks(c.L2T.nrows, c.plL2T.lanes), blocks(c.Yd.nrows, c.plY.lanes),
                                              blocks(c.YdT.nrows, c.plYT.lanes)});
    const int64_t nlong = std::max<int64_t>({(int64_t)c.plA.long_rows.size(), (int64_t)c.plAT.long_rows.size(),
                                             (int64_t)c.plL2.long_rows.size(), (int64_t)c.plL2T.long_rows.size(),
                                             (int64_t)c.plR.long_rows.size(), (int64_t)c.plRT.long_rows.size(),
                                             (int64_t)c.plY.long_rows.size(), (int64_t)c.plYT.long_rows.size()});
    L.npartials = (int32_t)(nparts + nlong + 64);
    L.partials = b.take(sizeof(double) * (size_t)L.npartials);
    int32_t nseg = std::max({(int32_t)c.plA.seg_beg.size(), (int32_t)c.plAT.seg_beg.size(),
                             (int32_t)c.plL2.seg_beg.size(), (int32_t)c.plL2T.seg_beg.size(),
                             (int32_t)c.plR.seg_beg.size(), (int32_t)c.plRT.seg_beg.size(),
                             (int32_t)c.plY.seg_beg.size(), (int32_t)c.plYT.seg_beg.size(), 1});
    L.nsegpart = nseg;
    L.segpart = b.take(sizeof(double) * (size_t)nseg);
    L.total = (b.off + 255) & ~(size_t)255;
}

}  // namespace rsilu
