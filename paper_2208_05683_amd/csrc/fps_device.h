// Internal declarations shared by the HIP kernels and the host library.
// Not part of the public ABI (include/fps.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fps {

constexpr int kWave = 64;
constexpr int kMaxTerms = 32;  // FPS_MAX_S + 1

// Summary of a stored row for the analysis, one 16-byte load: its entries,
// first and last column (first > last when empty), and its largest |value|
// rounded up to float (an upper bound of every |entry|).
struct __attribute__((aligned(16))) RowInfo {
    int32_t len;
    int32_t first;
    int32_t last;
    float amax;
};

// Row-range sparse matrix on the device.  Row r holds entries
// [beg[r], end[r]) of col/val, columns strictly increasing.  A canonical CSR
// is the special case end = row_ptr + 1.  info[r] summarises the row.
// Structure words: sw[beg[r] .. beg[r] + nw[r]) lists the row's columns by
// 32-column word, (column >> 5, bit (column & 31) set for each column of
// the row in that word), words ascending; nw[r] <= entries of the row.
struct MatView {
    const int64_t* beg;
    const int64_t* end;
    const int32_t* col;
    const double* val;
    const RowInfo* info;
    const uint2* sw;
    const int32_t* nw;
};

// Coefficient-sum operands: term t contributes coef[t] * M_t, with M_t the
// identity when beg[t] == nullptr.
struct Terms {
    int32_t n;
    double coef[kMaxTerms];
    const int64_t* beg[kMaxTerms];
    const int64_t* end[kMaxTerms];
    const int32_t* col[kMaxTerms];
    const double* val[kMaxTerms];
    const RowInfo* info[kMaxTerms];
    const uint2* sw[kMaxTerms];
    const int32_t* nw[kMaxTerms];
};

// Output of a stage in slack layout: row r may use [off[r], off[r+1]) and
// the kernel writes end[r] = off[r] + kept entries.
struct OutView {
    int64_t* off;  // n+1: row offsets (exclusive scan of the per-row upper bounds)
    int64_t* end;        // n
    int32_t* col;
    double* val;
    RowInfo* info;
    uint2* sw;    // structure words of row r at sw[off[r] ..]
    int32_t* nw;  // n: structure words of each row
    int64_t cap;  // capacity of col/val/sw
};

// Per-stage device counters (zeroed before each evaluation).  Only rare
// events use them; per-row statistics go to per-block partial sums (below)
// so that no hot path contends on one address.
struct StageCounters {
    unsigned long long fb_count;     // rows appended to the wide-tier list (fb_list)
    unsigned long long fb_next;      // dynamic fetch from fb_list, wide-tier kernel
    unsigned long long errors;       // bit flags, see kErr*
    unsigned long long kept_global;  // stored entries written by the wide-tier and device-memory kernels
    unsigned long long fb2_count;    // rows appended to the device-memory list (fb2_list)
    unsigned long long fb2_next;     // dynamic fetch from fb2_list, device-memory kernel
    unsigned long long rows_wide;    // rows computed by the wide-tier kernel
    unsigned long long max_ns;       // largest structural row computed by the wide-tier and device-memory kernels
    // dropped-entry statistics (only when StageArgs::dsum is set)
    unsigned long long n_dropped;       // nonzero entries removed by the tau test
    unsigned long long dropped_max;     // bits of the largest |dropped| (non-negative doubles order as integers)
    unsigned long long dropped_colmax;  // largest column sum of ceil(|dropped| * dscale)
};

// Algorithm 1 on the device (one record per state slot; three per stage: two
// alternating iteration states and the final record).
struct Alg1State {
    double t;      // threshold of the current iteration (the final one once done)
    double c;      // candidate norm of the final iteration
    int32_t it;    // iterations done
    int32_t done;  // the stopping test held
    int32_t ok;    // final record: 1 = converged within the launched iterations
    int32_t pad;
};

struct Alg1Params {
    double eps_g;   // filtering-norm threshold of the stage (finite, > 0)
    double target;  // eps_g (1 + e_r)
    double scale;   // 2^40 / eps_g
    int32_t max_iter;
    int32_t pad;
};

// Per-stage partial sums, one entry per block, layout [kPartCount][part_stride]:
// kPartMaxNs holds the largest structural row of the block and kPartMaxWords
// the widest window of its rows in 32-column words (maxima, not sums; the
// window width is written by the shared-memory tiers only).  kPartANnz is the
// product analysis' count of the left operand's stored entries in the block's
// rows (the dense-rows cost model reads it).  kPartBig counts the block's
// rows beyond the small-row tier (written by the 64-lane shared-memory
// kernels).
enum PartIndex : int {
    kPartProducts = 0,
    kPartProductsSkipped = 1,
    kPartRowsSkipped = 2,
    kPartKept = 3,
    kPartMaxNs = 4,
    kPartMaxWords = 5,
    kPartANnz = 6,
    kPartBig = 7,
    kPartCount = 8
};
constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each

constexpr unsigned long long kErrColumnOutsideWindow = 1;  // row summary inconsistent with data
constexpr unsigned long long kErrCapacity = 2;             // output total above capacity
constexpr unsigned long long kErrBadCsr = 4;               // validation failure
constexpr unsigned long long kErrNeedsGlobal = 8;          // a row needed the global-memory kernel that was not scheduled
constexpr unsigned long long kErrAlg1Pending = 16;         // Algorithm 1 needs more iterations than were launched

enum StageMode : int32_t { kModeProduct = 0, kModeSum = 1 };

// A stage computes, for every row r,
//     out_r = D_tau( extra_r + main_r )
// where main_r accumulates the terms of the stage (products A_rk B_k,: in
// product mode, c_t M_t[r,:] in coefficient-sum mode) and extra_r is either
// row r of E (has_e) or, in product mode with has_blk, the coefficient sum
// over T accumulated on its own (a coefficient block fused into a Horner
// step); without extra, out_r = D_tau(main_r).
struct StageArgs {
    int32_t mode;
    int32_t has_e;
    int32_t has_blk;
    int64_t n;
    double tau;
    double skip_tau;  // rows whose bound is below this are empty (0 disables the test)
    // Per-row thresholds (a batch of instances in one block-diagonal matrix):
    // when set, row r drops |x| < tau_row[r] instead of tau, and its empty-row
    // test uses tau_row[r] * skip_rel (skip_rel = 0 disables the test).
    const double* tau_row;
    double skip_rel;
    // when set, the analysis adds each computed row's multiply-adds to
    // prod_acc[r] (the batch autotuner's per-instance counts)
    int64_t* prod_acc;
    MatView A, B, E;
    Terms T;
    // analysis outputs
    int32_t* W;   // window width (0 = empty row)
    int32_t* lo;  // first column of the window
    int64_t* prod;  // entries of the row's main terms (0: the main part is empty)
    // Row offsets of the output: the analysis writes each row's offset within
    // its block of 2^scan_shift rows into out.off and the block totals into
    // blk_pre; a one-block scan turns blk_pre into the exclusive prefix of the
    // totals and writes out.off[n]; the numeric kernel adds
    // blk_pre[r >> scan_shift] to out.off[r] when it starts row r.
    int64_t* blk_pre;
    int32_t scan_shift;  // log2 of the rows per analysis block
    int32_t scan_pad;
    // > 0: row r of the output owns [r * row_stride, (r + 1) * row_stride)
    // instead (no scan of the analysis totals); the numeric kernel writes
    // out.off[r]
    int64_t row_stride;
    OutView out;
    StageCounters* ctr;
    const int32_t* dummy_col;  // 128 zeroed entries read by inactive lanes
    const double* dummy_val;
    unsigned long long* part;  // this stage's partial sums
    int64_t part_stride;
    int64_t* fb_list;       // n entries: rows for the wide shared-memory tier
    int64_t* fb2_list;      // n entries: rows for the device-memory kernel
    uint32_t* g_scratch;    // global-memory kernel workspace
    int64_t g_slot_words;   // bitmap words per slot (each array has room for one guard word / spare slot more)
    int64_t g_slot_cap;     // accumulator entries per slot
    int64_t g_slot_stride;  // 4-byte units between slots (multiple of 64)
    int64_t g_off_acc;      // 4-byte offsets of the slot's arrays: byte map at 0, bitmap words (uint2) at
    int64_t g_off_ebuf;     //   8 (words + 1), then accumulator and parked values
    int32_t g_slots;
    int32_t force_global;
    int32_t global_planned;  // 0: the device-memory kernel will not run for this stage
    int32_t wide_planned;    // 0: the wide-tier kernel will not run for this stage
    // The small-row tier computes each row's window, product count and
    // empty-row test itself (the analysis kernel is not launched; fixed row
    // strides only); the product counts then go to the partial sums at the
    // numeric kernel's four-row block index.
    int32_t fuse_analysis;
    // Column sums at the write-out: when dsum is set, every nonzero entry
    // removed by the tau test or with |x| <= dthr adds ceil(|x| * dscale) to
    // dsum[col] (exact integer sums); with dcount it is also counted in
    // ctr->n_dropped / ctr->dropped_max.  (Fixed threshold: the dropped-entry
    // statistics, dthr = 0.  Algorithm 1: the candidate sums of its first
    // iteration, dthr = eps_g.)
    unsigned long long* dsum;
    double dscale;
    double dthr;
    int32_t dcount;
    int32_t dpad;
};

// One instance of a batch as the join kernels read it: its canonical CSR
// (device), where its entries start in the joined matrix, and its threshold.
struct BatchSrc {
    const int64_t* row_ptr;
    const int32_t* col;
    const double* val;
    int64_t nnz_base;
    double tau;
};

// ---- launch wrappers (fps_batch.hip) ------------------------------------
// base[0..count]: first joined row of each instance (base[count] = total)
hipError_t launch_batch_join(const BatchSrc* src, const int64_t* base, int count, int64_t total, int64_t* rp,
                             int32_t* col, double* val, double* tau_row, hipStream_t s);
hipError_t launch_batch_bounds(const int64_t* frp, const int64_t* base, int count, int64_t* bounds, hipStream_t s);
// out[i] += sum of acc[r] over the rows of instance i (exact integer sums)
hipError_t launch_batch_instance_sum(const int64_t* acc, const int64_t* base, int count, int64_t total,
                                     unsigned long long* out, hipStream_t s);
hipError_t launch_batch_extract(const int64_t* frp, const int32_t* fcol, int64_t row0, int64_t n, int64_t p0,
                                int64_t cnt, int32_t shift, int64_t* rp, int32_t* col, hipStream_t s);

// ---- launch wrappers (fps_dense.hip) ------------------------------------
// leading dimension of the dense operands: n rounded up to 128
int64_t dense_ld(int64_t n);
// D = M as a dense ld x ld matrix, every entry written (zeros included)
hipError_t launch_densify(const MatView& M, int64_t n, int64_t ld, double* D, hipStream_t s);
// E = sum_t coef_t M_t in rows and columns < n, terms in order, one fma each
// from +0 (every such entry written, zeros included)
hipError_t launch_dense_terms(const Terms& T, int64_t n, int64_t ld, double* E, hipStream_t s);
// E = D_tau((has_e ? E : 0) + A B) on the matrix cores (tau per row if tau_row)
hipError_t launch_dgemm_mfma(const double* A, const double* B, double* E, int64_t ld, int64_t n, int has_e, double tau,
                             const double* tau_row, hipStream_t s);
// E = D_tau((has_e ? E : 0) + A B) on the vector units, each entry's sum over
// k in order (the sparse path's bits; ld a multiple of 128)
hipError_t launch_dgemm_ordered(const double* A, const double* B, double* E, int64_t ld, int64_t n, int has_e,
                                double tau, const double* tau_row, hipStream_t s);
// E = D_tau((has_e ? E : 0) + A B) with A sparse and B dense, each entry the
// fma chain over A's row in order (the sparse path's bits)
hipError_t launch_spmm_rows(const MatView& A, const double* B, double* E, int64_t ld, int64_t n, int has_e, double tau,
                            const double* tau_row, hipStream_t s);
// rows of the dense C written as the stage output a.out (placement, summaries,
// structure words, partial sums as the numeric kernels)
hipError_t launch_dense_to_slack(const double* C, int64_t ld, const StageArgs& a, hipStream_t s);

// ---- launch wrappers (fps_kernels.hip) ---------------------------------
// row summaries and the structure words (sw: nnz entries, nw: n) of a canonical CSR
hipError_t launch_rowinfo_csr(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t n,
                              RowInfo* info, uint2* sw, int32_t* nw, hipStream_t s);
hipError_t launch_validate_csr(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t n,
                               int64_t nnz, unsigned long long* err, hipStream_t s);
// the analysis of a stage, then (unless a.row_stride > 0) the scan of its
// block totals into row offsets
hipError_t launch_analyze(const StageArgs& a, hipStream_t s);
// log2 of the rows per analysis block (the numeric kernel's offset fix-up)
int analyze_shift(int32_t mode);
hipError_t launch_numeric_lds(const StageArgs& a, int grid, hipStream_t s);
// every row of the stage in the wide shared-memory tier (instead of
// launch_numeric_lds, for stages whose rows mostly exceed the narrow tier)
hipError_t launch_numeric_wide_rows(const StageArgs& a, hipStream_t s);
// Every row of a stage on a 16-lane DPP row (four rows per wavefront); rows
// beyond the tier go to the wide tier's list.  small_tier_fits tells
// whether a stage of n rows whose largest structural row and widest window
// (32-column words) are max_ns and max_words should run in the tier;
// small_tier_most, whether one with `big` rows beyond the tier should run
// there all the same (those rows then go to the wide tier).
hipError_t launch_numeric_small(const StageArgs& a, int64_t max_ns, int64_t max_words, hipStream_t s);
bool small_tier_fits(int64_t n, int64_t max_ns, int64_t max_words);
bool small_tier_most(int64_t n, int64_t big);
// rows of fb_list (persistent blocks: the grid size only sets the parallelism)
hipError_t launch_numeric_wide(const StageArgs& a, int grid, hipStream_t s);
// rows of fb2_list
hipError_t launch_numeric_global(const StageArgs& a, int grid, hipStream_t s);
// Canonical row pointers of a slack matrix: rp[r] gets the row's offset
// within its block of 256 rows, blk_pre the exclusive prefix of the block
// totals, rp[n] the total.  launch_compact adds the block prefix to rp[r]
// while it copies the rows.
hipError_t launch_row_offsets(const int64_t* beg, const int64_t* end, int64_t n, int64_t* rp, int64_t* blk_pre,
                              hipStream_t s);
// exclusive scan in place of nblk block totals, total to *grand (one block)
hipError_t launch_block_scan(int64_t* x, int64_t nblk, int64_t* grand, hipStream_t s);
hipError_t launch_compact(const int64_t* beg, const int64_t* end, const int32_t* col, const double* val,
                          int64_t n, int64_t* rp, const int64_t* blk_pre, int32_t* ocol, double* oval, hipStream_t s);
int64_t offset_blocks(int64_t n);
hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v, hipStream_t s);
int numeric_waves_per_block();
// Algorithm 1 helpers (adaptive filter)
hipError_t launch_alg1_colsum(const int64_t* beg, const int64_t* end, const int32_t* col, const double* val,
                              const RowInfo* info, int64_t n, double t, double scale, unsigned long long* colsum,
                              hipStream_t s);
hipError_t launch_max_u64(const unsigned long long* x, int64_t n, unsigned long long* out, hipStream_t s);
// (both drops also clear ctr->kept_global: they recount every row)
hipError_t launch_alg1_drop(const int64_t* beg, int64_t* end, int32_t* col, double* val, RowInfo* info,
                            uint2* sw, int32_t* nw, int64_t n, double t, unsigned long long* part_kept,
                            StageCounters* ctr, hipStream_t s);
// Algorithm 1 driven on the device: `iters` iteration kernels (state in
// st[0..1], column sums in cs[0..2n), maxima in cs[2n..2n+3), all zero on
// entry), then the final update and the drop; the final record goes to st[2];
// a stage that has not converged by then keeps its entries and raises
// kErrAlg1Pending in ctr->errors.
// (fused0: the numeric kernel already summed the first iteration's candidates
// into cs[0, n); finalize_only: the numeric kernel already dropped |x| <=
// t_dropped, and only the final state and flags are written, the evaluation
// being flagged for a repeat unless the iteration ends at t_dropped; base:
// column sums of those removed entries, with which every iteration's sums
// start, or null)
hipError_t launch_alg1_device(const int64_t* beg, int64_t* end, int32_t* col, double* val, RowInfo* info,
                              uint2* sw, int32_t* nw, int64_t n, const Alg1Params& pr, int iters, Alg1State* st, unsigned long long* cs,
                              unsigned long long* part_kept, StageCounters* ctr, int fused0, int finalize_only,
                              double t_dropped, const unsigned long long* base, hipStream_t s);
int numeric_global_blocks(int slots);
// blocks of the wide-tier kernel (persistent: six per CU at most)
int numeric_wide_blocks(int64_t n);
// 1-norm estimator (fps_normest.hip)
hipError_t launch_transpose(const int64_t* rp, const int32_t* col, const double* val, int64_t n, int64_t nnz,
                            unsigned long long* cnt, int64_t* trp, int32_t* trow_tmp, double* tval_tmp, int32_t* trow,
                            double* tval, hipStream_t s);
hipError_t launch_spmv(const int64_t* rp, const int32_t* col, const double* val, int64_t n, const double* x, double* y,
                       hipStream_t s);
// ||y||_1 = sum of |y_i| in ascending index order from +0 (one wavefront)
hipError_t launch_abs_sum_ordered(const double* y, int64_t n, double* out, hipStream_t s);
hipError_t launch_sign(const double* y, int64_t n, const double* s_old, int check, double* sv, unsigned int* flags,
                       hipStream_t s);
hipError_t launch_absmax(const double* h, int64_t n, unsigned long long* res, hipStream_t s);
hipError_t launch_fill_f64(double* x, int64_t n, double v, hipStream_t s);
hipError_t launch_unit_vector(double* x, int64_t n, int64_t i, hipStream_t s);
// number of blocks each kernel writes partials for (host-side reduction)
int64_t analyze_blocks(int32_t mode, int64_t n);
int64_t numeric_blocks(int64_t n);

}  // namespace fps
