// Internal declarations of the nAIR HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <initializer_list>
#include <string>
#include <vector>

#include "nair.h"

namespace nair {

constexpr int kMaxBs = 32;          // largest block size the kernels accept
constexpr int kMaxLevels = 64;
constexpr int kStallDenseDofs = 4096;
constexpr int kMaxGmres = 200;      // longest GMRES restart cycle
constexpr int kHashSmall = 2048;    // LDS hash slots of the per-wave symbolic kernels
constexpr int kHashLarge = 8192;    // LDS hash slots of the per-workgroup fallback

// ------------------------------------------------------------------ errors
struct Error {
    nair_status code;
    std::string msg;
};

// Throws nair::Error; caught at the ABI boundary.
[[noreturn]] void fail(nair_status code, const std::string &msg);
void check_hip(hipError_t e, const char *what);
#define NAIR_HIP(call) ::nair::check_hip((call), #call)

// ------------------------------------------------------------ device pool
// Caching device allocator: freed blocks are kept per size class for reuse,
// so repeated setups do not call hipMalloc.  Thread safe.
void *pool_alloc(size_t bytes);
void pool_free(void *p);
void pool_trim();
// A handle's caller-supplied allocator (nair_allocator).  While an AllocScope
// names one on a thread, pool_alloc takes device memory from it (for use on
// the scope's stream) instead of the pool; pool_free returns every block to
// where it came from, whatever scope is active then.
struct ExtAlloc {
    bool on = false;
    nair_allocator a{};
};
struct AllocScope {
    const ExtAlloc *prev;
    void *prev_stream;
    AllocScope(const ExtAlloc *e, void *stream);
    ~AllocScope();
};

template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        p = static_cast<T *>(pool_alloc(sizeof(T) * (count ? count : 1)));
    }
    void release() {
        if (p) pool_free(p);
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
};

// Device block-CSR matrix: nb rows, ncols block columns, bs x bs row-major blocks.
// nnzb < 0: the block count is only on the device (rowptr[nb]) and the arrays
// hold cap blocks; it is read back with a later synchronisation.
struct DevBSR {
    int nb = 0, ncols = 0, bs = 0;
    int64_t nnzb = 0;
    int64_t cap = 0;
    int64_t bound() const { return nnzb >= 0 ? nnzb : cap; }
    DBuf<int> rowptr, colidx;
    DBuf<double> vals;
    void alloc(int nb_, int ncols_, int bs_, int64_t nnzb_) {
        nb = nb_;
        ncols = ncols_;
        bs = bs_;
        nnzb = nnzb_;
        rowptr.alloc(static_cast<size_t>(nb_) + 1);
        colidx.alloc(static_cast<size_t>(nnzb_));
        vals.alloc(static_cast<size_t>(nnzb_) * bs_ * bs_);
    }
};

// ----------------------------------------------------------- kernel timer
enum TimedKernel { TK_RELAX = 0, TK_RESIDUAL = 1, TK_RESTRICT = 2, TK_INTERP = 3, TK_SPGEMM_NUM = 4,
                   TK_SPGEMM_SYM = 5, TK_BLOCKINV = 6, TK_RAP = 7, TK_DENSE = 8, TK_BLOCKPROD = 9 };
// Brackets launches of the selected (kernel, level) with events; no-ops otherwise.
struct TimerScope {
    bool on;
    hipStream_t s;
    // `launches`: number of back-to-back launches of the kernel inside the scope
    TimerScope(int kernel, int level, hipStream_t stream, int launches = 1);
    ~TimerScope();
};
void timer_select(int kernel, int level);
void timer_read(int64_t *launches, double *total_ms);
extern thread_local int g_timer_level;   // level the host code is working on
// Setup block products of 9x9, 16x16 and 25x25 blocks on the FP64 matrix cores
// (nair_params.matrix_cores, set per setup call); false: the vector-unit kernels.
extern thread_local bool g_matrix_cores;
inline bool use_matrix_cores(int bs) { return g_matrix_cores && (bs == 9 || bs == 16 || bs == 25); }
extern thread_local bool g_capturing;    // launches are being captured into a graph (timer off)
extern thread_local bool g_timer_off;    // the kernel timer skips these launches (no events are created)

// ------------------------------------------------------------- utilities
inline unsigned grid_for(int64_t n, int per_block) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 2147483647LL) g = 2147483647LL;
    return static_cast<unsigned>(g);
}

// Synchronous device-to-host reads (small ones staged through pinned memory;
// several items share one synchronisation).
struct ReadItem {
    const void *dev;
    void *host;
    size_t bytes;
};
void read_device(std::initializer_list<ReadItem> items, hipStream_t s);
void read_device(const ReadItem *items, size_t nitems, hipStream_t s);
int read_int(const int *dptr, hipStream_t s);
void read_ints(const int *dptr, int *host, int n, hipStream_t s);

// Exclusive scan of n ints: out[0..n], out[n] = total.  in may alias nothing in out.
// total_copy (nullable) receives the total too, so several totals can sit
// side by side and come back to the host in one copy
void scan_exclusive(const int *in, int *out, int n, hipStream_t s, int *total_copy = nullptr);
// Two scans in the same launches (lengths n0, n1; total0 / total1 as total_copy).
void scan_exclusive2(const int *in0, int *out0, int n0, int *total0, const int *in1, int *out1, int n1, int *total1,
                     hipStream_t s);

// ---------------------------------------------------------- setup kernels
void launch_block_maxabs(const double *vals, int64_t nnzb, int bs, double *out, hipStream_t s);
// Per block t < n (vals block src[t] if src, empty at or past *count if count):
// max-abs entry, nonzero rows | nonzero columns << 32, nonzero rows, and the
// nonzero rows times bs; each output may be null.  1 <= bs <= 32.  copy (nullable,
// no src or count): the blocks are also copied there, read once for both.
void launch_block_scan(const double *vals, int64_t n, int bs, const int *src, const int *count, double *maxabs,
                       uint64_t *meta, uint32_t *rmask, int *rsize, hipStream_t s, double *copy = nullptr);
// skip (nullable): blocks whose inverse is not needed (directly solved systems)
void launch_block_inverse(const int *rowptr, const int *colidx, const double *vals, int nb, int bs,
                          const int8_t *skip, double *dinv, int *singular_min, hipStream_t s);
// margin[0], margin[1] += comparisons within 1e-12 relative in the theta / phi tests
void launch_strength(const int *rowptr, const int *colidx, const double *bnorm, int nb, double theta,
                     double phi, uint8_t *mask, int *lambda, int *margin, hipStream_t s);
void launch_strong_transpose(const int *rowptr, const int *colidx, const uint8_t *mask, int nb,
                             const int *stptr, int *fill, int *stidx, hipStream_t s);
// splitting states: -1 undecided, 0 F, 1 C, 2 block of a directly solved system
void launch_pmis_init(const int *lambda, const int8_t *direct, int nb, int8_t *state, int *dround,
                      int *undecided0, hipStream_t s);
// lbase (nullable): first block of each block's system; hashes use the index within the system.
// undecided[0] receives the blocks still undecided after the round; when undecided[-1]
// (the previous round's count, or the start's) is 0 the round does nothing.
void launch_pmis_round(const int *rowptr, const int *colidx, const uint8_t *mask, const int *stptr,
                       const int *stidx, const int *lambda, const int *lbase, int nb, uint64_t seed, int level,
                       int round, int8_t *state, int8_t *newc, int *dround, int *undecided, hipStream_t s);
void launch_cf_flags(const int8_t *state, int nb, int want, int *flags, hipStream_t s);
// fscan (nullable): F-block exclusive scan when some blocks are neither F nor C
void launch_cf_index(const int8_t *cf, const int *cscan, const int *fscan, int nb, int *cidx, int *cpts,
                     int *flist, hipStream_t s);
// per block: lbase (first block of its system), direct (its system has mode 2), bsys (its system); each nullable
void launch_seg_info(const int *seg, const int8_t *mode, int nsys, int nb, int *lbase, int8_t *direct, int *bsys,
                     hipStream_t s);
void launch_mark_direct(const int8_t *direct, int nb, int8_t *state, hipStream_t s);
void launch_gather_int(const int *v, const int *idx, int n, int *out, hipStream_t s);
// p[i] = v for i < n, for up to four (p, n, v) arrays in one launch
struct FillInts {
    int *p;
    int64_t n;
    int v;
};
void launch_fill_ints(std::initializer_list<FillInts> jobs, hipStream_t s);
// margin[2] += F rows whose chosen C block has a rival within 1e-12 relative
void launch_one_point(const int *rowptr, const int *colidx, const double *bnorm, const int8_t *cf,
                      const int *cidx, int nb, int *pmap, int *margin, hipStream_t s);
// T = -(Dinv_I A_IJ) over phi-strong F-F blocks (fine row numbering, C rows empty)
void launch_count_T(const int *rowptr, const int *colidx, const uint8_t *mask, const int8_t *cf, int nb,
                    int *cnt, hipStream_t s);
void launch_fill_T(const int *rowptr, const int *colidx, const uint8_t *mask, const int8_t *cf, int nb,
                   const int *trowptr, int *tcol, int *trow, int *tsrc, hipStream_t s);
// W0 = A_cf (coarse rows)
void launch_count_Acf(const int *rowptr, const int *colidx, const int8_t *cf, const int *cpts, int nc,
                      int *cnt, hipStream_t s);
void launch_fill_Acf(const int *rowptr, const int *colidx, const int8_t *cf, const int *cpts, int nc,
                     const int *wrowptr, int *wcol, int *wsrc, hipStream_t s);
// out[t] = sign * (X[xi[t]] * Y[yi[t]]) for n blocks (fma chain, c ascending);
// count (device, nullable): only the first *count <= n blocks; rmask
// (nullable, 9x9 and 16x16 blocks): each product's nonzero rows as a bit mask
void launch_block_product(int64_t n, int bs, const double *X, const int *xi, const double *Y, const int *yi,
                          double sign, double *out, hipStream_t s, const int *count = nullptr,
                          uint32_t *rmask = nullptr);
// The terms of a sum of block matrices that is not stored: block t of the sum
// is the sum, in term order, of vals[i]'s block map[i][t] over the terms with
// map[i][t] >= 0 (the first present term, then each later one added to it: the
// order of repeated bsr_add).
constexpr int kMaxSumTerms = 17;   // Neumann degree 16 and W_0
struct SumTerms {
    const double *vals[kMaxSumTerms] = {};
    const int *map[kMaxSumTerms] = {};
    int n = 0;
};
// out[t] = sign * ((sum of the terms' blocks) * Y[yi[t]]) for the first *count
// <= n blocks of the sum's pattern, the sum added entry by entry as bsr_add adds
// it and the product formed as launch_block_product forms it (9x9, 16x16 and
// 25x25 blocks, matrix cores); rmask as there
void launch_sum_product(int64_t n, int bs, const SumTerms &terms, const double *Y, const int *yi, double sign,
                        double *out, hipStream_t s, const int *count, uint32_t *rmask);
// map[t] = map[t] >= 0 ? through[map[t]] : -1 for the first *count <= n entries
void launch_map_through(int64_t n, const int *count, int *map, const int *through, hipStream_t s);
// After O = S + W (pattern only, srcS from bsr_add): maps[i] (term i's block of
// each S block) become term i's block of each O block (-1 where srcS is -1),
// for the first *count <= cap blocks of O.
void compose_term_maps(int64_t cap, const int *count, const int *srcS, std::vector<DBuf<int>> &maps,
                       hipStream_t s);
// out[t] = Y[src[t]] for t < n (count, device, nullable: t < *count <= n)
void launch_block_gather(int64_t n, int bs, const double *Y, const int *src, double *out, hipStream_t s,
                         const int *count = nullptr);
void launch_rows_of(const int *rowptr, int nrows, int *rowid, hipStream_t s);

// ------------------------------------------------------------------ SpGEMM
// C = X * Y (+ optional implicit identity block of X at column xdiag[i]).
// Fixed accumulation order: inner index ascending, c ascending, one fma chain.
// (xmap: X's values are not stored with it; X's block x is block xmap[x] of xvals)
void spgemm(const DevBSR &X, const int *xdiag, const DevBSR &Y, DevBSR &C, hipStream_t s,
            const double *xvals = nullptr, const int *xmap = nullptr);
// O = S + W (union pattern, S's value first).  O's block count stays on the
// device (O.nnzb = -1, arrays of S.bound() + W.bound() blocks).
// With srcS and srcW given, only the pattern is formed: O.vals stays empty and
// block t of the sum is S's block (*srcS)[t] plus W's block (*srcW)[t] (-1:
// absent), for launch_sum_product.
void bsr_add(const DevBSR &S, const DevBSR &W, DevBSR &O, hipStream_t s, DBuf<int> *srcS = nullptr,
             DBuf<int> *srcW = nullptr);
// The Galerkin product K = R A P with R = [Z I] (identity at column cpts[i] of
// row i) and P one-point through pmap, filtered by drop.  K block (i, J) is the
// sum, in ascending fine column j, of the blocks (R A)_ij with pmap[j] = J, each
// (R A)_ij formed as in spgemm.  For 9x9 and 16x16 blocks the R A blocks are
// never stored: each K block is summed straight from their pair lists.
// margin[3] += off-diagonal blocks whose drop test is within 1e-12 relative;
// knext receives the block max-abs size of every kept block of K (the next
// level's block norms).  K's block count stays on the device (K.nnzb = -1,
// arrays of the unfiltered count).  A block count of Z left on the device is
// read back with the first synchronisation.
// kmask receives the row masks of K's kept blocks where the fused kernel forms
// them (9x9 and 16x16 blocks; left unallocated otherwise).
void galerkin(DevBSR &Z, const int *cpts, const DevBSR &A, const int *pmap, int nc, double drop, DevBSR &K,
              int *margin, DBuf<double> &knext, DBuf<uint32_t> &kmask, hipStream_t s);

// ------------------------------------------------------------------ dense
// For each segment k < nseg (host arrays): the dense operator of A's block rows
// [blk0[k], blk0[k] + nbk[k]) (no block outside the range), inverted into
// inv + off[k] and transposed into invT + off[k] (order n = nbk[k] * bs,
// row-major).  Returns -1, or the first segment whose operator is singular.
int dense_inverse_segments(const DevBSR &A, int nseg, const int *blk0_h, const int *nbk_h, const int64_t *off_h,
                           double *inv, double *invT, hipStream_t s);

// -------------------------------------------------------------- transpose
void bsr_transpose(const DevBSR &A, DevBSR &AT, hipStream_t s);   // blocks transposed too
void pmap_transpose(const int *pmap, int nb, int nc, DBuf<int> &ptptr, DBuf<int> &ptidx, hipStream_t s);

// ------------------------------------------------------------ face copy
// Compact copy of a BSR matrix whose off-diagonal blocks are nonzero only on a
// few rows and columns (upwind DG: the rows and columns of the two elements'
// nodes on the shared face).  Per block t, meta[t] holds the nonzero rows
// (bits 0..31) and nonzero columns (bits 32..63); its rmax x cmax rectangle
// vals[t * rc + p * cmax + q] holds the entry of its p-th nonzero row and q-th
// nonzero column (zero past its own counts).  Diagonal blocks (meta 0) are
// kept whole in dvals [nb][bs][bs] by columns (entry (a, c) at c * bs + a, so
// the lanes of a block row read consecutive words).  vals32 / dvals32: the
// same in float.
struct FaceCopy {
    bool on = false;
    int rmax = 0, cmax = 0, rc = 0;
    DBuf<uint64_t> meta;
    DBuf<double> vals, dvals;
    DBuf<float> vals32, dvals32;
};
// Build F for A when its off-diagonal blocks' nonzero rectangles hold at most
// half a block (F.on stays false otherwise).  Synchronises the stream once.
// (meta: the blocks' nonzero-row and nonzero-column masks when already known,
// taken over; else a pass over A's entries finds them)
void build_face(const DevBSR &A, FaceCopy &F, hipStream_t s, DBuf<uint64_t> *meta_known = nullptr);
void face_to_float(const DevBSR &A, FaceCopy &F, hipStream_t s);

// What the face-compressed kernels read (meta == nullptr: the plain BSR values).
template <typename MT>
struct FaceView {
    const uint64_t *meta = nullptr;
    const MT *vals = nullptr;
    const MT *dvals = nullptr;
    int cmax = 0, rc = 0;
};

// ------------------------------------------------------------ row blocks
// A list of bs x bs blocks stored by their nonzero rows: block t keeps the
// mask of its nonzero rows and those rows, whole and in ascending order, at
// vals[off[t]] ... (popcount(mask) * bs entries).  Z's blocks are nonzero only
// on the rows of the C element's nodes that face F neighbours.
struct RowBlocks {
    bool on = false;
    DBuf<uint32_t> mask;
    DBuf<int> off;   // [n + 1]
    DBuf<double> vals;
    DBuf<float> vals32;
};
// Blocks vals[src[d]] (src null: vals[d]) for d < *count (count null: n); the
// others are left empty.  Returns false (building nothing) when n * bs * bs
// exceeds int32 offsets.
// masks (nullable): the blocks' row masks, indexed like vals (read instead of the entries).
bool build_row_blocks(const double *vals, int64_t n, int bs, RowBlocks &R, hipStream_t s, const int *src = nullptr,
                      const int *count = nullptr, const uint32_t *masks = nullptr);
void row_blocks_to_float(RowBlocks &R, int64_t n, int bs, hipStream_t s);
template <typename MT>
struct RowBlockView {
    const uint32_t *mask = nullptr;   // null: whole blocks
    const int *off = nullptr;
    const MT *vals = nullptr;
};

// ------------------------------------------------------- transposed rows
// An operator M read as M^T for the transposed cycle, each block stored by M's
// nonzero rows: output row I (a block column of M) lists the blocks M_JI of the
// selected rows J of M in ascending J; entry t holds J, the mask of M_JI's
// nonzero rows and, at vals[off[t]] ..., those rows whole and in ascending
// order (popcount(mask) * bs entries, row-major).  Lane a of output row I then
// forms (M^T x)_I[a] = sum_t sum_k M_JI[c_k][a] x_J[c_k] over the nonzero rows
// c_k: consecutive lanes read consecutive words of a stored row, and the zero
// rows of M's blocks (most of a coarse block, all but the face rows of a DG
// face block) are neither stored nor read.  A whole transposed block would
// store every column of M's block as a row.  The products walk the stored rows
// flat: output row I owns stored rows qptr[I] .. qptr[I+1]-1 (entry by entry,
// each entry's rows in ascending c_k), and stored row q multiplies x at
// src[q] = J bs + c_k.
struct TransRows {
    bool on = false;
    int nrows = 0;                 // output rows (M's block columns)
    int64_t nent = 0;              // entries (blocks)
    int64_t nq = 0;                // stored rows
    DBuf<int> rowptr, colidx, off;
    DBuf<uint32_t> mask;
    DBuf<int> qptr, src;
    DBuf<double> vals;
    DBuf<float> vals32;
};
// M^T of M's blocks in rows J with keep_cf == null or cf[J] == keep_cf; mmask
// (nullable): the nonzero-row masks of M's blocks, else found from the values.
// Returns false (building nothing) when the kept rows exceed int32 offsets.
bool build_trans_rows(const DevBSR &M, const int8_t *cf, int keep_cf, const uint32_t *mmask, TransRows &T,
                      hipStream_t s);
void trans_rows_to_float(TransRows &T, int bs, hipStream_t s);
template <typename MT>
struct TransRowsView {
    int nrows = 0, bs = 0;
    int64_t nent = 0, nq = 0;
    const int *rowptr = nullptr, *colidx = nullptr, *off = nullptr;
    const uint32_t *mask = nullptr;
    const int *qptr = nullptr, *src = nullptr;
    const MT *vals = nullptr;
    int groups = 0;   // lane groups per output row (0: from the row length)
    TransRowsView with_groups(int g) const {
        TransRowsView v = *this;
        v.groups = g;
        return v;
    }
};

// ----------------------------------------------------------- sweep copy
// What a Jacobi F sweep reads, stored in the order it reads it: the F rows of
// a level operator (or of its transpose) in F-list order, each without its
// diagonal block, and D_F^{-1} in the same order with the coefficient of input
// c for output a at c * bs + a (D^{-1} transposed for the forward sweeps,
// D^{-1} itself for the transposed ones, which apply D^{-T}).  Row f (the F list's f-th
// row) holds blocks rowptr[f] .. rowptr[f+1]-1 in the row's ascending column
// order: by their nonzero rows (RowBlocks), or, where the operator has a
// face-compressed copy (rc > 0), that copy's masks and rmax x cmax rectangles.  Storage for
// vals and colidx is sized by the operator's block count (the exact count is
// rowptr[nF] on the device; nothing is read back).
struct SweepCopy {
    bool on = false;
    int nF = 0, cmax = 0, rc = 0;
    int64_t cap = 0;                 // blocks allocated
    DBuf<int> rowptr, colidx;
    DBuf<uint64_t> meta;
    DBuf<double> vals, dinv;
    DBuf<float> vals32;
    RowBlocks rows;                  // the blocks by their nonzero rows (no face copy)
};
// Build S from A (and its face copy F when F.on) for the rows of flist.
// amask (nullable): row masks of A's blocks.
// trans: the copy of A^T for the transposed sweeps (D^{-T} applied).
void build_sweep(const DevBSR &A, const FaceCopy &F, const double *dinv, const int *flist, int nF, SweepCopy &S,
                 hipStream_t s, bool trans, const uint32_t *amask = nullptr);
void sweep_to_float(SweepCopy &S, int bs, hipStream_t s);

template <typename MT>
struct SweepView {
    const int *rowptr = nullptr, *colidx = nullptr;
    const uint64_t *meta = nullptr;   // face rectangles when non-null
    const MT *vals = nullptr;
    const double *dinv = nullptr;
    int cmax = 0, rc = 0;
    RowBlockView<MT> rows{};          // else the blocks by their nonzero rows
};

// ------------------------------------------------------------------ cycle
// Read-only view of a BSR matrix with values of type MT (double, or float for
// the FP32-stored hierarchy), optionally with its face-compressed copy.
template <typename MT>
struct MatView {
    int nb = 0, ncols = 0, bs = 0;
    int64_t nnzb = 0;
    const int *rowptr = nullptr, *colidx = nullptr;
    const MT *vals = nullptr;
    int groups = 0;   // lane groups per block row for the kernel reading it (0: from the row length)
    FaceView<MT> face{};
    SweepView<MT> sweep{};   // F sweeps over the F list read this when rowptr != null
    RowBlockView<MT> rows{};   // the same blocks by their nonzero rows, when the level keeps them
    MatView with_groups(int g) const {
        MatView v = *this;
        v.groups = g;
        return v;
    }
};
inline MatView<double> view(const DevBSR &A) {
    return MatView<double>{A.nb, A.ncols, A.bs, A.nnzb, A.rowptr.get(), A.colidx.get(), A.vals.get(), 0};
}
inline MatView<float> view(const DevBSR &A, const float *vals32) {
    return MatView<float>{A.nb, A.ncols, A.bs, A.nnzb, A.rowptr.get(), A.colidx.get(), vals32, 0};
}
// lane-group counts a kernel may use for block size bs (powers of two, G * bs <= 256)
int max_groups(int bs);
// a level of `rows` block rows gives fewer than kFewLanes lanes at one group per
// row: its cycle kernels take more groups by default and are not tuned
constexpr int64_t kFewLanes = 32768;
bool few_lanes(int64_t rows, int bs);

// Rows of systems that have stopped iterating are skipped in batched solves:
// row r is live when active == nullptr or active[bsys ? bsys[r] : 0] != 0.
struct Gate {
    const int *bsys = nullptr;
    const int *active = nullptr;
};
__device__ inline bool live(const Gate &g, int row) {
    return g.active == nullptr || g.active[g.bsys ? g.bsys[row] : 0] != 0;
}

// r = b - A x (b == nullptr: r = A x), plus a float copy if r_lo
template <typename MT, typename VT>
void launch_residual(const MatView<MT> &A, const VT *b, const VT *x, VT *r, float *r_lo, hipStream_t s,
                     Gate g = Gate());
// Jacobi sweep over `list` rows (list == nullptr: all rows; then rows with cf != only_cf are copied)
template <typename MT, typename VT>
void launch_relax(const MatView<MT> &A, const double *dinv, bool dinv_trans, const VT *r, const VT *ein, VT *eout,
                  const int *list, int nlist, const int8_t *cf, int only_cf, hipStream_t s, Gate g = Gate());
// The first transposed F sweep from a zero guess: e1_F = D_F^{-T} r_F, other rows 0 in e0 and e1
template <typename VT>
void launch_relax_T_first(const double *dinv, const VT *r, const int8_t *cf, VT *e0, VT *e1, int nb, int bs,
                          hipStream_t s, Gate g = Gate());
// e0 = e1 = P e_c (one-point: block I takes e_c[pmap I], or zero)
template <typename VT>
void launch_interp(const int *pmap, const VT *ec, VT *e0, VT *e1, int nb, int bs, hipStream_t s, Gate g = Gate());
// gate of the coarse rows (coarse-level system ids)
template <typename MT, typename VT>
void launch_restrict(const MatView<MT> &Z, const VT *r, const int *cpts, VT *rc, hipStream_t s, Gate g = Gate());
template <typename VT>
void launch_restrict_T(const int *ptptr, const int *ptidx, const VT *s, VT *sc, int nc, int bs, hipStream_t st,
                       Gate g = Gate());
// e0 = P e_c everywhere, e1 = e0 + D^{-1}(r - A e0) on F rows (e0 on C rows):
// the interpolation and the first F sweep in one launch
template <typename MT, typename VT>
void launch_relax_interp(const MatView<MT> &A, const double *dinv, const VT *r, const int *pmap, const VT *ec,
                         const int8_t *cf, VT *e0, VT *e1, hipStream_t s, Gate gate = Gate());
template <typename MT, typename VT>
void launch_interp_T(const MatView<MT> &ZT, const int *cidx, const VT *yc, VT *y, hipStream_t s, Gate g = Gate());
// The transposed cycle's products read from TransRows copies (coarse levels):
// s = g - A^T y on every row, with y zero outside the copy's source rows
template <typename MT, typename VT>
void launch_residual_tr(const TransRowsView<MT> &T, const VT *g, const VT *y, VT *sout, hipStream_t s,
                        Gate gate = Gate());
// transposed Jacobi F sweep over `list`: y_out_I = D_I^{-T}(g_I - sum_{J != I} (A^T)_IJ y_in_J)
template <typename MT, typename VT>
void launch_sweep_tr(const TransRowsView<MT> &T, const double *dinv, const VT *g, const VT *yin, VT *yout,
                     const int *list, int nlist, hipStream_t s, Gate gate = Gate());
// y_I += [I is C] yc_{cidx I} + (Z^T yc)_I
template <typename MT, typename VT>
void launch_interp_tr(const TransRowsView<MT> &T, const int *cidx, const VT *yc, VT *y, hipStream_t s,
                      Gate gate = Gate());
template <typename VT>
void launch_init_T(const double *dinv, const VT *g, const int8_t *cf, int fc, VT *y0, VT *y1, int nb, int bs,
                   hipStream_t s, Gate gate = Gate());
template <typename VT>
void launch_axpy(double *x, const VT *e, int64_t n, hipStream_t s);
// y_k = M_k x_k for nseg dense segments: M_k at M + off[k], order n[k], vectors at dof0[k];
// segments of stopped systems (active[sys[k]] == 0; active nullable) are skipped
template <typename VT>
void launch_dense_matvec(const double *M, const int64_t *off, const int *dof0, const int *n, int nseg, int max_n,
                         const VT *x, VT *y, hipStream_t s, const int *sys = nullptr, const int *active = nullptr);
// dst = src / dst += src on the block rows of live systems
template <typename VT>
void launch_copy_vec(VT *dst, const VT *src, int nb, int bs, hipStream_t s, Gate g = Gate());
template <typename VT>
void launch_add_vec(VT *dst, const VT *src, int nb, int bs, hipStream_t s, Gate g = Gate());
// x += e on the dofs of systems still iterating (active[bsys[block]]; bsys == nullptr: system 0)
template <typename VT>
void launch_axpy_active(double *x, const VT *e, int64_t n, int bs, const int *bsys, const int *active,
                        hipStream_t s);
// per-chunk sums of squares (chunk c: dofs [clo[c], clo[c] + clen[c]))
void launch_seg_sumsq(const double *v, const int64_t *clo, const int *clen, int nchunk, double *part,
                      hipStream_t s);
// start of a batched solve: per-system ||b|| from the chunk sums; activity, status, counters
// (nact_acc: a scratch counter)
void launch_seg_init(const double *part, const int *cptr, int nsys, double *bn, double *last, int *active,
                     int *status, int *iters, int *it, int *nact, int *nact_acc, hipStream_t s);
// end of one batched iteration: per-system relative residual, history, convergence, counters
void launch_seg_check(const double *part, const int *cptr, int nsys, const double *bn, const double *rtol,
                      int hist_cap, double *hist, double *last, int *active, int *status, int *iters, int *it,
                      int *nact, int *nact_acc, hipStream_t s);
// out[i] = (float) in[i] for i < n (count, device, nullable: i < min(n, *count))
void launch_to_float(const double *in, float *out, int64_t n, hipStream_t s, const int *count = nullptr);

// ------------------------------------------------------------ scalar form
// S = D^{-1} A as a scalar matrix (bs 1): identity diagonal blocks exact,
// off-diagonal blocks D_I^{-1} A_IJ (fma chains), exact zeros dropped.
void build_scaled(const DevBSR &A, const double *dinv, DevBSR &S, hipStream_t s);
// out (and out32 if given) = D^{-1} v blockwise (trans: D^{-T} v), rows of live systems
template <typename VT>
void launch_block_diag_apply(const double *dinv, const VT *v, double *out, float *out32, int nb, int bs, bool trans,
                             hipStream_t s, Gate g = Gate());

// ----------------------------------------------------------------- Krylov
// V holds nv vectors of n doubles, vector i at V + i * ld.
// out[i] = <V_i, w> for i < nv (part: mdot_parts(n) * nv doubles of scratch).
// Deterministic: fixed chunks, fixed reduction order.
int64_t mdot_parts(int64_t n);
void launch_mdot(const double *V, int64_t ld, int nv, const double *w, int64_t n, double *part, double *out,
                 hipStream_t s);
// w -= sum_i c[i] V_i, i ascending (c on the device)
void launch_maxpy(const double *V, int64_t ld, int nv, const double *c, double *w, int64_t n, hipStream_t s);
// v = w / sqrt(*ss) (device scalar)
void launch_unit(const double *w, const double *ss, double *v, int64_t n, hipStream_t s);

// ------------------------------------------------------------------- grad
void grad_vals(int nb, int bs, const int *rowptr, const int *colidx, const double *ybar, const double *x,
               double *gvals, hipStream_t s);

}  // namespace nair
