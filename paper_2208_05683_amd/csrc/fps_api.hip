// Host side of libfps: plans, the stage schedule of Algorithm 2 (fixed tau),
// device buffers, and the C ABI declared in include/fps.h.
#include "fps.h"
#include "fps_device.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace fps;

namespace {

thread_local std::string g_last_error;

fps_status set_error(fps_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                                          \
    do {                                                                                                       \
        hipError_t e_ = (expr);                                                                                \
        if (e_ != hipSuccess) {                                                                                \
            (void)hipGetLastError();                                                                           \
            return set_error(e_ == hipErrorOutOfMemory ? FPS_ERR_OUT_OF_MEMORY : FPS_ERR_HIP, "%s: %s (%s:%d)", \
                             #expr, hipGetErrorString(e_), __FILE__, __LINE__);                                \
        }                                                                                                      \
    } while (0)

#define FPS_TRY(expr)                      \
    do {                                   \
        fps_status s_ = (expr);            \
        if (s_ != FPS_OK) return s_;       \
    } while (0)

// Device bytes held by one owner (a plan), with an optional limit.  The
// owner makes its account current on the calling thread (AcctScope) for the
// duration of each entry point; allocations made meanwhile are charged to
// it and fail with FPS_ERR_CAPACITY past the limit.
struct MemAcct {
    size_t used = 0;
    size_t peak = 0;
    size_t cap = SIZE_MAX;
    // optional: asked to raise `cap` to at least `need` before an allocation
    // past it fails (true if it did)
    bool (*extend)(void* ctx, MemAcct* a, size_t need) = nullptr;
    void* ctx = nullptr;
    // room for `more` bytes beside `used`, after asking for it if needed
    bool admit(size_t more)
    {
        if (more <= cap && used <= cap - more) return true;
        return extend != nullptr && used <= SIZE_MAX - more && extend(ctx, this, used + more) && more <= cap &&
               used <= cap - more;
    }
};
thread_local MemAcct* t_acct = nullptr;

// A stage's rows get a fixed stride when that takes at most this many times
// the room of the scanned upper bounds.
constexpr int64_t kStrideRoom = 4;

struct AcctScope {
    MemAcct* prev;
    explicit AcctScope(MemAcct* a) : prev(t_acct) { t_acct = a; }
    ~AcctScope() { t_acct = prev; }
};

// Device buffers recycled without hipMalloc / hipFree (a hipFree
// synchronises the whole device, which would serialise concurrent requests).
// Used by the server's worker threads, where every buffer is released only
// after the stream that used it has been synchronised (and a result only
// after the copies out of it have finished), so a block handed out again is
// never still in use.  Sizes are rounded up to classes of 4 KiB below
// 64 KiB, else to the next 2^k or 1.5 * 2^k.
struct DevPool {
    std::mutex mu;
    std::multimap<size_t, void*> free_blocks;
    size_t cached = 0;  // bytes of the free blocks

    static size_t size_class(size_t b)
    {
        if (b <= (size_t(64) << 10)) return (b + 4095) / 4096 * 4096;
        size_t p = size_t(1) << (63 - __builtin_clzll((unsigned long long)b));
        if (p == b) return b;
        return (b <= p + p / 2) ? p + p / 2 : 2 * p;
    }
    void* take(size_t cls)
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = free_blocks.find(cls);
        if (it == free_blocks.end()) return nullptr;
        void* p = it->second;
        free_blocks.erase(it);
        cached -= cls;
        return p;
    }
    void give(void* p, size_t cls)
    {
        std::lock_guard<std::mutex> lk(mu);
        free_blocks.emplace(cls, p);
        cached += cls;
    }
    // hipFree free blocks (largest first) until at most `keep` bytes are cached
    void trim(size_t keep)
    {
        std::lock_guard<std::mutex> lk(mu);
        while (cached > keep && !free_blocks.empty()) {
            auto it = std::prev(free_blocks.end());
            (void)hipFree(it->second);
            cached -= it->first;
            free_blocks.erase(it);
        }
    }
    ~DevPool() { trim(0); }
};
thread_local DevPool* t_pool = nullptr;

// Grow-only device allocation (from the calling thread's pool if it has one).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    MemAcct* acct = nullptr;  // the account charged for p
    DevPool* pool = nullptr;  // the pool p came from (it goes back there)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) {
            if (pool)
                pool->give(p, bytes);
            else
                (void)hipFree(p);
            if (acct) acct->used -= bytes;
        }
        p = nullptr;
        bytes = 0;
        acct = nullptr;
        pool = nullptr;
    }
    fps_status ensure(size_t want)
    {
        if (want <= bytes && p) return FPS_OK;
        release();
        size_t b = std::max<size_t>(want, 256);
        if (t_pool) b = DevPool::size_class(b);
        if (t_acct && !t_acct->admit(b))
            return set_error(FPS_ERR_CAPACITY, "device memory limit of %zu bytes reached (%zu held, %zu more wanted)",
                             t_acct->cap, t_acct->used, b);
        p = t_pool ? t_pool->take(b) : nullptr;
        if (!p) {
            hipError_t e = hipMalloc(&p, b);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                p = nullptr;
                return set_error(FPS_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) failed: %s", b, hipGetErrorString(e));
            }
        }
        bytes = b;
        pool = t_pool;
        acct = t_acct;
        if (acct) {
            acct->used += b;
            acct->peak = std::max(acct->peak, acct->used);
        }
        return FPS_OK;
    }
    template <typename T>
    T* as() const
    {
        return static_cast<T*>(p);
    }
};

// A stage output in slack layout (see OutView).
struct SlackMatrix {
    int64_t n = 0;
    int64_t cap = 0;
    DevBuf off, end, info, col, val, sw, nw;
    fps_status ensure_rows(int64_t nn)
    {
        n = nn;
        FPS_TRY(off.ensure(sizeof(int64_t) * (size_t)(nn + 1)));
        FPS_TRY(end.ensure(sizeof(int64_t) * (size_t)std::max<int64_t>(nn, 1)));
        FPS_TRY(info.ensure(sizeof(RowInfo) * (size_t)std::max<int64_t>(nn, 1)));
        FPS_TRY(nw.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nn, 1)));
        return FPS_OK;
    }
    fps_status ensure_cap(int64_t c)
    {
        if (c <= cap && col.p) return FPS_OK;
        const int64_t want = std::max<int64_t>(c + c / 8, 64);
        FPS_TRY(col.ensure(sizeof(int32_t) * (size_t)want));
        FPS_TRY(val.ensure(sizeof(double) * (size_t)want));
        FPS_TRY(sw.ensure(sizeof(uint2) * (size_t)want));
        cap = want;
        return FPS_OK;
    }
    MatView view() const
    {
        return MatView{off.as<int64_t>(), end.as<int64_t>(), col.as<int32_t>(), val.as<double>(), info.as<RowInfo>(),
                       sw.as<uint2>(), nw.as<int32_t>()};
    }
    OutView out() const
    {
        return OutView{off.as<int64_t>(), end.as<int64_t>(), col.as<int32_t>(), val.as<double>(), info.as<RowInfo>(),
                       sw.as<uint2>(), nw.as<int32_t>(), cap};
    }
};

// A canonical CSR owned by the library.
struct CanonMatrix {
    int64_t n = 0;
    int64_t cap = 0;
    DevBuf rp, col, val;
};

// Algorithm 1 on the device: the first iteration's column sums taken in the
// numeric kernel's write-out.
constexpr bool kAlg1FuseFirst = true;
// ... and, for stages that needed one iteration, the drop applied there too.
constexpr bool kAlg1DropFirst = true;
// ... and, for stages that needed more, the drop at the learned final threshold.
constexpr bool kAlg1DropLearned = true;

// Per-row workspace shared by the stages of one engine.
struct Workspace {
    int64_t n = 0;
    DevBuf W, lo, ub, fb, fb2, blk_pre, zinfo, zsw, znw, gscratch, counters, part, dummy, dsum;
    int64_t g_words = 0, g_cap = 0, g_stride = 0, g_off_acc = 0, g_off_ebuf = 0;
    int64_t part_stride = 0;
    int32_t g_slots = 0;
    int max_stages = 0;

    fps_status init(int64_t nn, int stages, hipStream_t st)
    {
        n = nn;
        max_stages = stages;
        const size_t rows = (size_t)std::max<int64_t>(nn, 1);
        FPS_TRY(W.ensure(sizeof(int32_t) * rows));
        FPS_TRY(lo.ensure(sizeof(int32_t) * rows));
        FPS_TRY(ub.ensure(sizeof(int64_t) * rows));
        FPS_TRY(fb.ensure(sizeof(int64_t) * rows));
        FPS_TRY(fb2.ensure(sizeof(int64_t) * rows));
        FPS_TRY(blk_pre.ensure(sizeof(int64_t) * (size_t)(std::max({analyze_blocks(kModeProduct, nn),
                                                                    analyze_blocks(kModeSum, nn),
                                                                    offset_blocks(nn)}) + 1)));
        FPS_TRY(zinfo.ensure(sizeof(RowInfo) * rows));
        FPS_TRY(znw.ensure(sizeof(int32_t) * rows));
        FPS_TRY(counters.ensure(sizeof(StageCounters) * (size_t)stages));
        FPS_TRY(dummy.ensure(128 * (sizeof(int32_t) + sizeof(double))));
        HIP_TRY(launch_fill_u64(dummy.as<unsigned long long>(), 128 * (sizeof(int32_t) + sizeof(double)) / 8, 0ull, st));
        part_stride = std::max({analyze_blocks(kModeProduct, nn), analyze_blocks(kModeSum, nn), numeric_blocks(nn)}) + 1;
        FPS_TRY(part.ensure(sizeof(unsigned long long) * (size_t)(kPartCount * part_stride * stages)));
        // global-memory kernel: per slot byte map + bitmap + prefix + accumulator for a full row
        g_words = (nn + 31) / 32;
        g_cap = std::max<int64_t>(nn, 1);
        // per slot (4-byte units): byte map and guard word [8 (words + 1)] | bitmap words as uint2 and
        // the guard word [2 (words + 1)] | accumulator and the spare slot [2 (cap + 1)] | parked
        // values [2 cap]
        g_off_acc = 10 * (g_words + 1);
        g_off_ebuf = g_off_acc + 2 * (g_cap + 1);
        const int64_t per_slot_u32 = (g_off_ebuf + 2 * g_cap + 63) / 64 * 64;
        g_stride = per_slot_u32;
        // up to 2048 wavefronts (eight per CU) with a workspace each, 4 GiB at most
        const int64_t budget = int64_t(1) << 32;
        int64_t slots = std::min<int64_t>(2048, std::max<int64_t>(4, budget / (4 * per_slot_u32)));
        slots = std::min<int64_t>(slots, std::max<int64_t>(4, ((nn + 3) / 4) * 4));
        slots = (slots + numeric_waves_per_block() - 1) / numeric_waves_per_block() * numeric_waves_per_block();
        g_slots = (int32_t)slots;
        return FPS_OK;  // the device-memory kernel's workspace: ensure_global, when a stage needs it
    }

    // The device-memory kernel's per-wavefront workspace, allocated the
    // first time a stage sends rows to that kernel (most plans never do).
    fps_status ensure_global()
    {
        return gscratch.ensure(sizeof(uint32_t) * (size_t)g_stride * (size_t)g_slots);
    }
};

// Largest n (exclusive) for the exact integer column sums of Algorithm 1.
constexpr int64_t kColSumMaxN = int64_t(1) << 24;

enum class Kind { Power = FPS_STAGE_POWER, Block = FPS_STAGE_BLOCK, GStep = FPS_STAGE_GSTEP, Horner = FPS_STAGE_HORNER };

constexpr int kTimingRing = 64;   // sampled evaluations whose kernel times are kept
// the dense path a product stage takes (fps_stats.stage_dense)
constexpr int kDenseNone = 0, kDenseMfma = 1, kDenseRows = 2, kDenseOrdered = 3;

constexpr int kTimingEvery = 8;   // every 8th evaluation records events (each record costs a few microseconds)

struct StageRecord {
    int kind = 0, index = 0;
    int a_src = -1, b_src = -1, e_src = -1;  // stage that produced the operand (-1: Z or none)
    bool a_is_z = false, b_is_z = false;
    std::vector<int> term_src;  // coefficient sums: per matrix term, -1 = Z, else producing stage
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // events of the current evaluation (ring slot)
    // adaptive filter (Algorithm 1) of this stage
    double eps_g = 0.0, threshold = 0.0, dropped = 0.0;
    int alg1_iters = 0;
    bool alg1_device = false;  // the record is in the device state (Engine::alg1_state)
    int alg1_mode = 0;         // fps_stats.stage_alg1_mode
    bool wide_rows = false;    // every row of the stage ran in the wide shared-memory tier
    bool small = false;        // every row of the stage ran in the small-row tier (four rows per wavefront)
    int dense = 0;             // the dense path the product ran on (kDenseNone, kDenseMfma, kDenseRows)
};

struct Schedule {
    int N = 0, q = 0, b = 0, g = 0, J = 0, start = 0, nsp = 0;
};

bool make_schedule(int m, int s, Schedule* sc)
{
    if (m < 0 || s < 1) return false;
    sc->N = m + 1;
    sc->q = s;
    sc->b = (sc->N + s - 1) / s;
    sc->g = (sc->N - sc->q * (sc->b - 1) == 1) ? 1 : 0;
    sc->J = (sc->b >= 2) ? sc->q : m;
    sc->start = (sc->b >= 2) ? 1 + sc->g : 0;
    sc->nsp = (sc->J >= 1 ? sc->J - 1 : 0) + (sc->b >= 2 ? sc->b - 1 - sc->g : 0);
    return true;
}

// Filtering-norm thresholds of eq. 28 for a polynomial of known degree: zeta_k
// for the powers (k = 2..q) and sigma_j for the Horner steps, from d_k
// (eq. 24), beta (eq. 21) and the norm bounds of eqs. 25-26, with z[t] >=
// ||Z^t||.  Sums run in ascending index order with separate multiplications
// and additions; M = number of filtered stages; a zero d_k is replaced by 1.
void fnt_thresholds(const std::vector<double>& c, int m, const Schedule& sc, double eps, const std::vector<double>& z,
                    std::vector<double>& zeta, std::vector<double>& sigma)
{
    const int q = sc.q, b = sc.b;
    auto A = [&](int k) { return (k >= 0 && k <= m) ? std::fabs(c[(size_t)k]) : 0.0; };
    std::vector<double> nb((size_t)b), ns((size_t)b);
    for (int i = 0; i < b; ++i) {
        double acc = 0.0;
        for (int j = 0; j < q; ++j) acc = acc + A(i * q + j) * z[(size_t)j];
        nb[(size_t)i] = acc;
    }
    ns[0] = nb[(size_t)(b - 1)];
    for (int i = 1; i < b; ++i) ns[(size_t)i] = nb[(size_t)(b - 1 - i)] + z[(size_t)q] * ns[(size_t)(i - 1)];
    const double M = (double)(sc.nsp > 0 ? sc.nsp : 1);
    zeta.assign((size_t)q + 1, INFINITY);
    for (int k = 2; k <= q; ++k) {
        double d = 0.0;
        for (int j = 0; j < b; ++j) {
            const int i = b - 1 - j;
            double beta = 0.0;
            if (k < q)
                for (int kk = k; kk < q; ++kk) beta = beta + A(i * q + kk) * z[(size_t)(kk - k)];
            const double sprev = (j >= 1) ? ns[(size_t)(j - 1)] : 0.0;
            d = d + z[(size_t)(q * (b - 1 - j))] * (beta + z[(size_t)(q - k)] * sprev);
        }
        if (d == 0.0) d = 1.0;
        zeta[(size_t)k] = eps / (d * M);
    }
    sigma.assign((size_t)b, 0.0);
    for (int j = 0; j < b; ++j) sigma[(size_t)j] = eps / (z[(size_t)(q * (b - 1 - j))] * M);
}

// Runs row-accumulation stages with one workspace.

struct Engine {
    Workspace ws;
    DevBuf colsum;  // Algorithm 1 column sums (two buffers) and maxima
    DevBuf alg1st;  // per stage: two Algorithm 1 iteration states and the final record
    uint64_t flags = 0;
    std::vector<int64_t> learned;  // per stage index: output capacity learned by a sizing run
    std::vector<int64_t> learned_ns;  // per stage index: largest structural row seen by a sizing run
    std::vector<int64_t> learned_words;  // per stage index: widest row window (32-column words) seen by a sizing run
    std::vector<int64_t> learned_big;    // per stage index: rows beyond the small-row tier in a sizing run
    std::vector<int64_t> learned_stride;  // per stage index: fixed row stride chosen by a sizing run (0: scanned)
    std::vector<int> fused;  // per stage index: the last run did the analysis in the small-row kernel
    std::vector<int64_t> learned_wide;    // per stage: rows a sizing run sent to the wide shared-memory tier
    std::vector<int64_t> learned_global;  // per stage: rows a sizing run sent to the device-memory kernel
    std::vector<int> alg1_learned;  // per stage: Algorithm 1 iterations of the last host-driven run
    std::vector<double> alg1_learned_t;  // ... and its final threshold
    // dense paths (FPS_FLAG_DENSE, FPS_FLAG_DENSE_EXACT): per stage the decision
    // of the sizing run (kDenseNone, kDenseMfma, kDenseRows, kDenseOrdered); three dense
    // ld x ld operands; which left operand dA holds (its column
    // array) and for which evaluation (P_q is the left operand of every
    // Horner step of an evaluation, densified once)
    std::vector<int> learned_dense;
    DevBuf dA, dB, dE;
    int64_t d_ld = 0;
    const void* dA_key = nullptr;
    int64_t dA_eval = -1, eval_id = 0;

    StageCounters* ctr(int i) const { return ws.counters.as<StageCounters>() + i; }
    Alg1State* alg1_state(int i) const { return alg1st.as<Alg1State>() + 3 * (size_t)i; }
    unsigned long long* part(int i) const
    {
        return ws.part.as<unsigned long long>() + (size_t)i * kPartCount * (size_t)ws.part_stride;
    }

    // Host reduction of a stage's per-block partial sums.
    fps_status stage_totals(int i, int32_t mode, unsigned long long out[kPartCount])
    {
        const int64_t na = analyze_blocks(mode, ws.n), nk = numeric_blocks(ws.n);
        std::vector<unsigned long long> h((size_t)(kPartCount * ws.part_stride));
        HIP_TRY(hipMemcpy(h.data(), part(i), sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
        for (int k = 0; k < kPartCount; ++k) {
            const bool per_row_block = k == kPartKept || k == kPartMaxNs || k == kPartMaxWords || k == kPartBig ||
                                       (fused[(size_t)i] && k <= kPartRowsSkipped);
            const bool maximum = k == kPartMaxNs || k == kPartMaxWords;
            const int64_t cnt = per_row_block ? nk : na;
            unsigned long long t = 0;
            for (int64_t b = 0; b < cnt; ++b) {
                const unsigned long long v = h[(size_t)(k * ws.part_stride + b)];
                t = maximum ? std::max(t, v) : t + v;
            }
            out[k] = t;
        }
        StageCounters c{};
        HIP_TRY(hipMemcpy(&c, ctr(i), sizeof(c), hipMemcpyDeviceToHost));
        out[kPartKept] += c.kept_global;
        out[kPartMaxNs] = std::max(out[kPartMaxNs], c.max_ns);
        return FPS_OK;
    }

    fps_status init(int64_t n, int stages, uint64_t fl, hipStream_t st)
    {
        flags = fl;
        learned.assign((size_t)stages, -1);
        learned_ns.assign((size_t)stages, 0);
        learned_words.assign((size_t)stages, 0);
        learned_big.assign((size_t)stages, 0);
        learned_stride.assign((size_t)stages, 0);
        fused.assign((size_t)stages, 0);
        learned_wide.assign((size_t)stages, 0);
        learned_global.assign((size_t)stages, 0);
        alg1_learned.assign((size_t)stages, 0);
        alg1_learned_t.assign((size_t)stages, 0.0);
        learned_dense.assign((size_t)stages, 0);
        FPS_TRY(alg1st.ensure(sizeof(Alg1State) * 3 * (size_t)std::max(stages, 1)));
        return ws.init(n, stages, st);
    }

    // A stage's output bound (measured by its analysis in a sizing run) must
    // fit the free device memory (either path writes its rows there); if it
    // does not, the evaluation stops with FPS_ERR_CAPACITY and the footprint,
    // the dense path's three operands included (the fill has outgrown the GPU).
    fps_status fits_device(int idx, int64_t total, bool product)
    {
        const double per_entry = sizeof(int32_t) + sizeof(double) + sizeof(uint2);  // column, value, word
        const double need = per_entry * (double)total;
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            return FPS_OK;  // no information: let the allocation decide
        }
        const double ld = (double)dense_ld(ws.n);
        const double dense_need = 3.0 * ld * ld * 8.0;
        if (need <= 0.95 * (double)fr) return FPS_OK;
        (void)product;
        return set_error(FPS_ERR_CAPACITY,
                         "stage %d: the output bound of %lld entries (%.0f per row, measured by the analysis) needs "
                         "%.1f GB; the dense path needs %.1f GB; %.1f GB of %.1f GB are free",
                         idx, (long long)total, (double)total / (double)std::max<int64_t>(ws.n, 1), need / 1e9,
                         dense_need / 1e9, (double)fr / 1e9, (double)tot / 1e9);
    }

    // Whether a product stage goes to the dense path: the modelled time of
    // the dense product is below that of the sparse one, and three dense
    // operands fit the free device memory (and the plan's limit).  Sparse:
    // the analysis' multiply-adds at the measured rate of the row kernel the
    // rows will take (2.5e11 per second in shared memory, 5e10 in the
    // device-memory kernel for rows beyond 512 entries on average); dense:
    // 2 ld^3 flops at 5e13 per second on the matrix cores (4.9e13 measured at
    // ld = 1024, 6.5e13 at 8064), four passes over ld^2 doubles at 4 TB/s
    // (densify, Bhat, the product's and the slack write-outs) and 10 us of
    // launches.
    // The path of a product stage by modelled time: sparse = the analysis'
    // multiply-adds at the rate of the row kernel its rows take (2.5e11/s in
    // shared memory, 5e10/s in the device-memory kernel, measured); matrix
    // cores = 2 ld^3 at 5e13 flop/s plus four passes over ld^2 doubles; the
    // ordered product on the vector units = 2 ld^3 at 3e13 flop/s plus five
    // passes; dense rows = one row of B (ld doubles) streamed per stored entry
    // of A at 4 TB/s plus four passes.  The matrix cores only with
    // FPS_FLAG_DENSE, the two exact paths with either flag; each needs its
    // operands' memory.
    int want_dense(int idx, int64_t bound_total, hipStream_t s)
    {
        unsigned long long prods = 0, a_nnz = 0;
        {
            const int64_t na = analyze_blocks(kModeProduct, ws.n);
            std::vector<unsigned long long> h((size_t)(kPartCount * ws.part_stride));
            if (hipMemcpyAsync(h.data(), part(idx), sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost,
                               s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                (void)hipGetLastError();
                return kDenseNone;
            }
            for (int64_t b = 0; b < na; ++b) {
                prods += h[(size_t)(kPartProducts * ws.part_stride + b)];
                a_nnz += h[(size_t)(kPartANnz * ws.part_stride + b)];
            }
        }
        const double ld = (double)dense_ld(ws.n);
        const double per_row = (double)bound_total / (double)std::max<int64_t>(ws.n, 1);
        const double t_sparse = (double)prods / (per_row > 512.0 ? 5e10 : 2.5e11);
        const double t_mfma = (flags & FPS_FLAG_DENSE) ? 2.0 * ld * ld * ld / 5e13 + 4.0 * ld * ld * 8.0 / 4e12 + 10e-6
                                                        : HUGE_VAL;
        const double t_rows = (double)a_nnz * ld * 8.0 / 4e12 + 4.0 * ld * ld * 8.0 / 3e12 + 20e-6;
        const double t_ordered = 2.0 * ld * ld * ld / 3e13 + 5.0 * ld * ld * 8.0 / 3e12 + 20e-6;
        int mode = kDenseMfma;
        double t_best = t_mfma;
        if (t_ordered < t_best) {
            mode = kDenseOrdered;
            t_best = t_ordered;
        }
        if (t_rows < t_best) {
            mode = kDenseRows;
            t_best = t_rows;
        }
        if (t_best >= t_sparse) return kDenseNone;
        // operands: B and E, and A densified for the dense products
        const double ops = mode == kDenseRows ? 2.0 : 3.0;
        const double need = ops * ld * ld * 8.0 - (double)(dA.bytes + dB.bytes + dE.bytes);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            return kDenseNone;
        }
        if (need > 0.9 * (double)fr) return kDenseNone;
        if (t_acct && t_acct->used + (size_t)std::max(0.0, need) > t_acct->cap) return kDenseNone;
        return mode;
    }

    // The product of stage `a` on the dense path into `out` (see
    // launch_dgemm_mfma): operands densified, Bhat formed densely, the
    // product with the block and the filter in its write-out, rows written
    // back as slack CSR.
    fps_status run_dense(StageArgs& a, int mode, hipStream_t s)
    {
        const int64_t n = ws.n, ld = dense_ld(n);
        const size_t bytes = sizeof(double) * (size_t)ld * (size_t)ld;
        FPS_TRY(dB.ensure(bytes));
        FPS_TRY(dE.ensure(bytes));
        if (ld != d_ld) dA_key = nullptr;
        d_ld = ld;
        if (mode == kDenseRows) {
            // A stays sparse: its rows stream B's dense rows in term order
            HIP_TRY(launch_densify(a.B, n, ld, dB.as<double>(), s));
            if (a.has_blk) HIP_TRY(launch_dense_terms(a.T, n, ld, dE.as<double>(), s));
            HIP_TRY(launch_spmm_rows(a.A, dB.as<double>(), dE.as<double>(), ld, n, a.has_blk, a.tau, a.tau_row, s));
            HIP_TRY(launch_dense_to_slack(dE.as<double>(), ld, a, s));
            return FPS_OK;
        }
        FPS_TRY(dA.ensure(bytes));
        if (!(dA_key == a.A.col && dA_eval == eval_id)) {
            HIP_TRY(launch_densify(a.A, n, ld, dA.as<double>(), s));
            dA_key = a.A.col;
            dA_eval = eval_id;
        }
        HIP_TRY(launch_densify(a.B, n, ld, dB.as<double>(), s));
        if (a.has_blk) HIP_TRY(launch_dense_terms(a.T, n, ld, dE.as<double>(), s));  // (every entry written)
        if (mode == kDenseOrdered)
            HIP_TRY(launch_dgemm_ordered(dA.as<double>(), dB.as<double>(), dE.as<double>(), ld, n, a.has_blk, a.tau,
                                         a.tau_row, s));
        else
            HIP_TRY(launch_dgemm_mfma(dA.as<double>(), dB.as<double>(), dE.as<double>(), ld, n, a.has_blk, a.tau,
                                      a.tau_row, s));
        HIP_TRY(launch_dense_to_slack(dE.as<double>(), ld, a, s));
        return FPS_OK;
    }

    // The row placement of stage idx after its sizing run: a fixed stride (the
    // largest structural row rounded up to 16 entries, at least 16) when that
    // takes no more room than the scanned row bounds, or up to kStrideRoom
    // times that room if the extra device memory is at hand (a quarter of the
    // free memory, within the plan's limit); else 0, scanned offsets.
    // Output buffers that the stride needs larger than the sizing run left
    // them are grown at the end of the sizing evaluation (once its work is
    // done), so that the evaluation after it allocates nothing.
    std::vector<std::pair<SlackMatrix*, int64_t>> grow_after_sizing;
    bool one_shot = false;  // the plan is evaluated once (a served request): nothing to prepare
    void decide_stride(int idx, SlackMatrix& out, int64_t n)
    {
        learned_stride[(size_t)idx] = 0;
        if (one_shot) return;
        const int64_t ns_max = learned_ns[(size_t)idx];
        const int64_t stride = std::max<int64_t>(16, (ns_max + 15) / 16 * 16);
        const int64_t bound = learned[(size_t)idx] / std::max<int64_t>(n, 1);
        bool ok = ns_max == 0 || stride <= bound;
        if (!ok && stride <= kStrideRoom * bound) {
            const double per_entry = sizeof(int32_t) + sizeof(double) + sizeof(uint2);  // column, value, word
            const double extra = per_entry * (double)std::max<int64_t>(0, stride * n - out.cap);
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
                (void)hipGetLastError();
                fr = 0;
            }
            ok = extra <= 0.25 * (double)fr && (!t_acct || (double)t_acct->used + extra <= (double)t_acct->cap);
        }
        if (!ok) return;
        learned_stride[(size_t)idx] = stride;
        if (stride * n > out.cap) grow_after_sizing.emplace_back(&out, stride * n);
    }
    fps_status grow_for_strides(hipStream_t s)
    {
        if (grow_after_sizing.empty()) return FPS_OK;
        HIP_TRY(hipStreamSynchronize(s));  // the buffers' sizing contents are no longer read
        for (auto& g : grow_after_sizing) FPS_TRY(g.first->ensure_cap(g.second));
        grow_after_sizing.clear();
        return FPS_OK;
    }

    // Runs one stage into `out`.  With `size` true the stream is synchronised to
    // read the output bound and the buffers are grown to fit; otherwise the
    // capacities learned earlier are used as they are.
    fps_status run(int idx, StageArgs& a, SlackMatrix& out, hipStream_t s, bool size, StageRecord* rec)
    {
        const int64_t n = ws.n;
        a.n = n;
        a.W = ws.W.as<int32_t>();
        a.lo = ws.lo.as<int32_t>();
        a.prod = ws.ub.as<int64_t>();
        a.ctr = ctr(idx);
        a.part = part(idx);
        a.dummy_val = ws.dummy.as<double>();
        a.dummy_col = reinterpret_cast<const int32_t*>(ws.dummy.as<double>() + 128);
        a.part_stride = ws.part_stride;
        a.fb_list = ws.fb.as<int64_t>();
        a.fb2_list = ws.fb2.as<int64_t>();
        a.g_scratch = ws.gscratch.as<uint32_t>();
        a.g_slot_words = ws.g_words;
        a.g_slot_cap = ws.g_cap;
        a.g_slot_stride = ws.g_stride;
        a.g_off_acc = ws.g_off_acc;
        a.g_off_ebuf = ws.g_off_ebuf;
        a.g_slots = ws.g_slots;
        a.force_global = (flags & FPS_FLAG_FORCE_GLOBAL) ? 1 : 0;
        FPS_TRY(out.ensure_rows(n));
        a.blk_pre = ws.blk_pre.as<int64_t>();
        a.scan_shift = analyze_shift(a.mode);
        const bool sizing = size || learned[(size_t)idx] < 0;
        // After sizing, rows get a fixed stride (the largest structural row
        // seen, rounded up to 16 entries, at least 16) when that takes at most
        // kStrideRoom times the room of the scanned upper bounds (rows of
        // uneven length, as in a joined batch, still qualify), or when every
        // row was empty: no offsets scan, and the small-row tier can take the
        // row's analysis into its own kernel.
        a.row_stride = sizing ? 0 : learned_stride[(size_t)idx];
        FPS_TRY(out.ensure_cap(a.row_stride > 0 ? a.row_stride * n : std::max<int64_t>(learned[(size_t)idx], 0)));
        a.out = out.out();  // the analysis writes the row offsets (out.off)
        // a stage whose sizing run kept every row within the small-row tier
        // runs four rows per wavefront; with fixed row strides that kernel
        // also does each row's analysis (no analysis launch, no offsets
        // scan).  (Taking the analysis into the 64-lane kernel as well made
        // its long rows slower than the separate launch costs.)
        const bool wide_rows = !sizing && !a.force_global && learned_wide[(size_t)idx] * 8 > n;
        // (or, with fixed row strides, most of them: the others, which the
        // sizing run counted, go on to the wide tier)
        const bool small_all = small_tier_fits(n, learned_ns[(size_t)idx], learned_words[(size_t)idx]);
        const bool small = !sizing && !wide_rows && !a.force_global && !a.has_e && !(flags & FPS_FLAG_NO_SMALL) &&
                           !learned_dense[(size_t)idx] && learned_wide[(size_t)idx] == 0 &&
                           learned_global[(size_t)idx] == 0 &&
                           (small_all || (a.row_stride > 0 && small_tier_most(n, learned_big[(size_t)idx])));
        const int64_t small_deferred = (small && !small_all) ? learned_big[(size_t)idx] : 0;
        a.fuse_analysis = (small && a.row_stride > 0 && a.prod_acc == nullptr) ? 1 : 0;
        fused[(size_t)idx] = a.fuse_analysis;
        if (!a.fuse_analysis) HIP_TRY(launch_analyze(a, s));
        // fallback kernels: a sizing run launches each one when rows reached
        // its list (read back after the kernel before it); later runs launch
        // those that a sizing run needed, with grids for the rows seen then
        // (their blocks fetch rows until the list is exhausted, so any grid
        // is correct; every wavefront of the grid takes one fetch ticket)
        bool run_wide = true, run_global = true;
        if (sizing) {
            int64_t total = 0;
            HIP_TRY(hipMemcpyAsync(&total, out.off.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            FPS_TRY(fits_device(idx, total, a.mode == kModeProduct));
            FPS_TRY(out.ensure_cap(total));
            learned[(size_t)idx] = std::max<int64_t>(learned[(size_t)idx], total);
        } else {
            run_wide = (learned_wide[(size_t)idx] > 0 || small_deferred > 0) && !a.force_global;
            run_global = learned_global[(size_t)idx] > 0 || a.force_global;
        }
        // a dense path for a product stage whose work has gone dense
        int dense = kDenseNone;
        // (not with dropped-entry statistics; Algorithm 1's first-iteration
        // sums, without a drop, the dense write-out takes as well)
        const bool sums_only =
            a.dsum != nullptr && a.dcount == 0 && a.dthr > 0.0 && a.tau == 0.0 && a.tau_row == nullptr;
        if (a.mode == kModeProduct && !a.has_e && (flags & (FPS_FLAG_DENSE | FPS_FLAG_DENSE_EXACT)) &&
            (a.dsum == nullptr || sums_only)) {
            if (sizing) learned_dense[(size_t)idx] = want_dense(idx, learned[(size_t)idx], s);
            dense = learned_dense[(size_t)idx];
        }
        if (rec) rec->dense = dense;
        if (dense != kDenseNone) {
            a.out = out.out();
            if (rec && rec->ev0) HIP_TRY(hipEventRecord(rec->ev0, s));
            FPS_TRY(run_dense(a, dense, s));
            if (rec && rec->ev1) HIP_TRY(hipEventRecord(rec->ev1, s));
            if (sizing) {
                unsigned long long tot[kPartCount];
                FPS_TRY(stage_totals(idx, a.mode, tot));
                learned_ns[(size_t)idx] = std::max<int64_t>(learned_ns[(size_t)idx], (int64_t)tot[kPartMaxNs]);
                decide_stride(idx, out, n);
            }
            return FPS_OK;
        }
        // a stage whose sizing run sent more than an eighth of its rows past the
        // narrow tier runs every row in the wide tier (instead of building
        // those rows' structure twice)
        if (wide_rows) run_wide = false;
        if (rec) rec->wide_rows = wide_rows;
        if (rec) rec->small = small;
        a.out = out.out();
        a.wide_planned = run_wide ? 1 : 0;
        a.global_planned = run_global ? 1 : 0;
        const int64_t per_block = numeric_waves_per_block();
        auto grid_for_rows = [&](int64_t rows, int64_t cap) {
            return (int)std::max<int64_t>(1, std::min<int64_t>((rows + per_block - 1) / per_block, cap));
        };
        if (rec && rec->ev0) HIP_TRY(hipEventRecord(rec->ev0, s));
        if (small)
            HIP_TRY(launch_numeric_small(a, learned_ns[(size_t)idx], learned_words[(size_t)idx], s));
        else if (wide_rows)
            HIP_TRY(launch_numeric_wide_rows(a, s));
        else
            HIP_TRY(launch_numeric_lds(a, 0, s));
        // (without sizing the stage's numeric kernels are timed together: the
        // end event follows the fallback tiers below)
        if (sizing && rec && rec->ev1) HIP_TRY(hipEventRecord(rec->ev1, s));
        StageCounters c{};
        if (sizing) {
            HIP_TRY(hipMemcpyAsync(&c, ctr(idx), sizeof(c), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            learned_wide[(size_t)idx] = std::max<int64_t>(learned_wide[(size_t)idx], (int64_t)c.fb_count);
            run_wide = c.fb_count > 0;
        }
        if (run_wide)
            HIP_TRY(launch_numeric_wide(
                a, grid_for_rows(std::max(learned_wide[(size_t)idx], small_deferred), numeric_wide_blocks(n)), s));
        if (sizing) {
            HIP_TRY(hipMemcpyAsync(&c, ctr(idx), sizeof(c), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            learned_global[(size_t)idx] = std::max<int64_t>(learned_global[(size_t)idx], (int64_t)c.fb2_count);
            run_global = c.fb2_count > 0;
        }
        if (run_global) {
            FPS_TRY(ws.ensure_global());
            a.g_scratch = ws.gscratch.as<uint32_t>();
        }
        if (run_global)
            HIP_TRY(launch_numeric_global(
                a, grid_for_rows(std::max<int64_t>(learned_global[(size_t)idx], a.force_global ? n : 0),
                                 numeric_global_blocks(ws.g_slots)),
                s));
        if (!sizing && rec && rec->ev1) HIP_TRY(hipEventRecord(rec->ev1, s));
        if (sizing) {
            // the stage's largest structural row
            unsigned long long tot[kPartCount];
            FPS_TRY(stage_totals(idx, a.mode, tot));
            learned_ns[(size_t)idx] = std::max<int64_t>(learned_ns[(size_t)idx], (int64_t)tot[kPartMaxNs]);
            learned_words[(size_t)idx] = std::max<int64_t>(learned_words[(size_t)idx], (int64_t)tot[kPartMaxWords]);
            learned_big[(size_t)idx] = std::max<int64_t>(learned_big[(size_t)idx], (int64_t)tot[kPartBig]);
            decide_stride(idx, out, n);
        }
        return FPS_OK;
    }

    // Algorithm 1 on a stage output in place (see fps_plan_create_ex).
    // device_iters > 0: that many iterations are launched as kernels (no host
    // round trip; the record is read back with the statistics); a stage that
    // needs more raises kErrAlg1Pending and the evaluation is repeated with the
    // host loop.  device_iters == 0: the count learned by the last host-driven
    // run of this stage, or the host loop (which learns it) if there is none.
    // device_iters < 0: the host loop, one synchronisation per iteration.
    // Before a stage that Algorithm 1 will filter on the device: the numeric
    // kernel's write-out sums the first iteration's candidates (0 < |x| <=
    // eps_g, the first threshold) into the column sums, which saves that
    // iteration's pass over the product.
    // When the stage needed a single iteration before (the count learned by
    // the host loop), the write-out also drops those candidates at once, as
    // that iteration would if its candidate norm is within the target; the
    // final state is then only checked on the device, and a miss raises
    // kErrAlg1Pending like any other iteration count that falls short.
    // With more iterations learned, the final threshold t* learned with them
    // is applied at the write-out in the same way: the removed entries' column
    // sums D go to a buffer of their own, every iteration sums the kept
    // entries below its threshold on top of D (exact while its threshold is
    // at least t*, which holds up to the first threshold below t*), and the
    // evaluation is flagged for a repeat unless the iteration ends at t*.
    int alg1_fused = 0;  // 0: not fused, 1: first iteration's sums, 2: sums and drop, 3: drop at t*
    double alg1_spec_t = 0.0;
    fps_status alg1_fuse(int idx, double eps_g, int device_iters, StageArgs& a, hipStream_t s)
    {
        alg1_fused = 0;
        if (device_iters == 0) device_iters = alg1_learned[(size_t)idx];
        if (device_iters <= 0 || !std::isfinite(eps_g) || !(eps_g > 0.0) || !kAlg1FuseFirst) return FPS_OK;
        // a stage on a dense path takes the first iteration's sums only (its
        // product's write-out applies the stage's own threshold, which must
        // then keep every nonzero)
        const bool dense = learned_dense[(size_t)idx] != kDenseNone;
        if (dense && (a.tau != 0.0 || a.tau_row != nullptr)) return FPS_OK;
        const int64_t n = ws.n;
        FPS_TRY(colsum.ensure(sizeof(unsigned long long) * (size_t)(3 * n + 3)));
        unsigned long long* cs = colsum.as<unsigned long long>();
        const double t_learned = alg1_learned_t[(size_t)idx];
        const bool spec = !dense && device_iters >= 2 && kAlg1DropLearned && t_learned > 0.0 && t_learned < eps_g;
        HIP_TRY(launch_fill_u64(cs, (spec ? 3 : 2) * n + 3, 0ull, s));
        a.dscale = std::ldexp(1.0, 40) / eps_g;
        a.dcount = 0;
        if (!dense && device_iters == 1 && kAlg1DropFirst) {
            // keep |x| > eps_g: !(|x| < tau) with tau the next double above eps_g
            a.dsum = cs;
            a.tau = std::nextafter(eps_g, HUGE_VAL);
            a.skip_tau = 0.0;
            a.dthr = 0.0;  // the summed entries are exactly the removed ones
            alg1_fused = 2;
            alg1_spec_t = eps_g;
        } else if (spec) {
            a.dsum = cs + 2 * n + 3;  // D
            a.tau = std::nextafter(t_learned, HUGE_VAL);
            a.skip_tau = 0.0;
            a.dthr = 0.0;
            alg1_fused = 3;
            alg1_spec_t = t_learned;
        } else {
            a.dsum = cs;
            a.dthr = eps_g;
            alg1_fused = 1;
        }
        return FPS_OK;
    }

    fps_status alg1(int idx, SlackMatrix& out, double eps_g, double e_r, int max_iter, hipStream_t s,
                    StageRecord* rec, int device_iters)
    {
        const int fused = alg1_fused;
        alg1_fused = 0;
        if (device_iters == 0) device_iters = alg1_learned[(size_t)idx];  // 0 if none: host loop

        const int64_t n = ws.n;
        if (rec) {
            rec->eps_g = eps_g;
            rec->threshold = 0.0;
            rec->dropped = 0.0;
            rec->alg1_iters = 0;
            rec->alg1_device = false;
            rec->alg1_mode = 0;
        }
        if (!std::isfinite(eps_g)) return FPS_OK;  // an unbounded budget filters nothing
        FPS_TRY(colsum.ensure(sizeof(unsigned long long) * (size_t)(2 * n + 3)));
        unsigned long long* cs = colsum.as<unsigned long long>();
        unsigned long long* mx = cs + n;
        const double target = eps_g * (1.0 + e_r);
        const double scale = std::ldexp(1.0, 40) / eps_g;
        if (device_iters > 0) {
            device_iters = std::min(device_iters, max_iter);
            if (fused == 2) device_iters = 1;
            if (!fused) HIP_TRY(launch_fill_u64(cs, 2 * n + 3, 0ull, s));
            const unsigned long long* base = nullptr;
            if (fused == 3) {  // the first iteration's sums start from D as well
                base = cs + 2 * n + 3;
                HIP_TRY(hipMemcpyAsync(cs, base, sizeof(unsigned long long) * (size_t)n, hipMemcpyDeviceToDevice, s));
            }
            const Alg1Params pr{eps_g, target, scale, max_iter, 0};
            HIP_TRY(launch_alg1_device(out.off.as<int64_t>(), out.end.as<int64_t>(), out.col.as<int32_t>(),
                                       out.val.as<double>(), out.info.as<RowInfo>(),
                                       out.sw.as<uint2>(), out.nw.as<int32_t>(), n, pr,
                                       device_iters, alg1_state(idx),
                                       cs, part(idx) + (size_t)kPartKept * (size_t)ws.part_stride, ctr(idx),
                                       (fused == 1 || fused == 2) ? 1 : 0, fused >= 2 ? 1 : 0, alg1_spec_t, base,
                                       s));
            if (rec) {
                rec->alg1_device = true;
                rec->alg1_mode = fused ? fused : 4;
            }
            return FPS_OK;
        }
        double m = 1.0, t = 0.0, c = 0.0;
        int it = 0;
        do {
            t = eps_g / m;
            HIP_TRY(launch_fill_u64(cs, n + 1, 0ull, s));
            HIP_TRY(launch_alg1_colsum(out.off.as<int64_t>(), out.end.as<int64_t>(), out.col.as<int32_t>(),
                                       out.val.as<double>(), out.info.as<RowInfo>(), n, t, scale, cs, s));
            HIP_TRY(launch_max_u64(cs, n, mx, s));
            unsigned long long h = 0;
            HIP_TRY(hipMemcpyAsync(&h, mx, sizeof(h), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            c = (double)h / scale;
            m = c / t;
            ++it;
        } while (c > target && it < max_iter);
        if (c > target)
            return set_error(FPS_ERR_CAPACITY, "Algorithm 1 did not reach its target within %d iterations", max_iter);
        HIP_TRY(launch_alg1_drop(out.off.as<int64_t>(), out.end.as<int64_t>(), out.col.as<int32_t>(),
                                 out.val.as<double>(), out.info.as<RowInfo>(),
                                 out.sw.as<uint2>(), out.nw.as<int32_t>(), n, t,
                                 part(idx) + (size_t)kPartKept * (size_t)ws.part_stride, ctr(idx), s));
        if (rec) {
            rec->threshold = t;
            rec->dropped = c;
            rec->alg1_iters = it;
        }
        alg1_learned[(size_t)idx] = it;
        alg1_learned_t[(size_t)idx] = t;
        return FPS_OK;
    }

    // Canonical compaction of a slack matrix.
    fps_status compact(const SlackMatrix& m, CanonMatrix& c, hipStream_t s)
    {
        const int64_t n = m.n;
        c.n = n;
        FPS_TRY(c.rp.ensure(sizeof(int64_t) * (size_t)(n + 1)));
        // room for every entry m can hold, now and (after a sizing run) with
        // the capacity its fixed stride will give it, so that the evaluations
        // after the sizing one do not grow the result
        int64_t want = std::max<int64_t>(m.cap, 1);
        for (const auto& g : grow_after_sizing)
            if (g.first == &m) want = std::max(want, g.second + g.second / 8);
        if (want > c.cap) {
            FPS_TRY(c.col.ensure(sizeof(int32_t) * (size_t)want));
            FPS_TRY(c.val.ensure(sizeof(double) * (size_t)want));
            c.cap = want;
        }
        HIP_TRY(launch_row_offsets(m.off.as<int64_t>(), m.end.as<int64_t>(), n, c.rp.as<int64_t>(),
                                   ws.blk_pre.as<int64_t>(), s));
        HIP_TRY(launch_compact(m.off.as<int64_t>(), m.end.as<int64_t>(), m.col.as<int32_t>(), m.val.as<double>(), n,
                               c.rp.as<int64_t>(), ws.blk_pre.as<int64_t>(), c.col.as<int32_t>(),
                               c.val.as<double>(), s));
        return FPS_OK;
    }
};

fps_status check_view(const fps_csr_view* v, const char* what, int64_t n_expect)
{
    if (!v) return set_error(FPS_ERR_INVALID_ARG, "%s is NULL", what);
    if (v->n < 1 || v->n > FPS_MAX_N) return set_error(FPS_ERR_INVALID_ARG, "%s: n = %lld out of range", what, (long long)v->n);
    if (n_expect >= 0 && v->n != n_expect) return set_error(FPS_ERR_INVALID_ARG, "%s: dimension mismatch", what);
    if (v->nnz < 0) return set_error(FPS_ERR_INVALID_ARG, "%s: negative nnz", what);
    if (!v->row_ptr || (v->nnz > 0 && (!v->col || !v->val)))
        return set_error(FPS_ERR_INVALID_ARG, "%s: null device pointer", what);
    return FPS_OK;
}

// Checks a CSR view on the device; the error flag lives in `flag` (8 bytes of
// device memory) when given, else in a buffer allocated here.
fps_status validate_on_device(const fps_csr_view* v, const char* what, hipStream_t s,
                              unsigned long long* flag = nullptr)
{
    DevBuf err;
    if (!flag) {
        FPS_TRY(err.ensure(sizeof(unsigned long long)));
        flag = err.as<unsigned long long>();
    }
    HIP_TRY(launch_fill_u64(flag, 1, 0ull, s));
    HIP_TRY(launch_validate_csr(v->row_ptr, v->col, v->val, v->n, v->nnz, flag, s));
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h) return set_error(FPS_ERR_BAD_CSR, "%s is not a canonical CSR (row pointers, sorted in-range columns, finite values)", what);
    return FPS_OK;
}

// ---- 1-norm estimator and norm bounds (series mode, Section 3.2.2) --------------

// Device workspace of the estimator on Z: Z^T as a CSR whose rows list the
// rows of Z in ascending order, and the vectors of the iteration.  The pieces
// are carved from one region, either owned by the workspace or given by the
// caller (fps_normest1_noalloc), at 256-byte boundaries.
constexpr size_t est_align(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t est_bytes(int64_t n, int64_t nnz)
{
    const size_t nn = (size_t)(n > 0 ? n : 1), nz = (size_t)(nnz > 0 ? nnz : 1);
    return est_align(sizeof(int64_t) * (nn + 1)) + 2 * est_align(sizeof(int32_t) * nz) +
           2 * est_align(sizeof(double) * nz) + est_align(sizeof(unsigned long long) * nn) +
           7 * est_align(sizeof(double) * nn) + est_align(64);
}

struct EstWork {
    int64_t n = 0;
    DevBuf own;
    int64_t* trp = nullptr;
    int32_t *trow = nullptr, *trow_tmp = nullptr;
    double *tval = nullptr, *tval_tmp = nullptr;
    unsigned long long* cnt = nullptr;
    double *x = nullptr, *y = nullptr, *t0 = nullptr, *t1 = nullptr, *s = nullptr, *s_old = nullptr, *zt = nullptr;
    char* small = nullptr;

    fps_status init(const fps_csr_view* Z, hipStream_t st)
    {
        FPS_TRY(own.ensure(est_bytes(Z->n, Z->nnz)));
        return init_at(Z, own.p, st);
    }

    // Carves the workspace from `base` (est_bytes(n, nnz) bytes of device
    // memory) and builds Z^T there; allocates nothing.
    fps_status init_at(const fps_csr_view* Z, void* base, hipStream_t st)
    {
        n = Z->n;
        const size_t nn = (size_t)n, nz = (size_t)std::max<int64_t>(Z->nnz, 1);
        char* c = static_cast<char*>(base);
        auto take = [&](size_t bytes) {
            char* r = c;
            c += est_align(bytes);
            return r;
        };
        trp = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (nn + 1)));
        trow = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nz));
        trow_tmp = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * nz));
        tval = reinterpret_cast<double*>(take(sizeof(double) * nz));
        tval_tmp = reinterpret_cast<double*>(take(sizeof(double) * nz));
        cnt = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * nn));
        for (double** v : {&x, &y, &t0, &t1, &s, &s_old, &zt}) *v = reinterpret_cast<double*>(take(sizeof(double) * nn));
        small = take(64);
        HIP_TRY(launch_transpose(Z->row_ptr, Z->col, Z->val, n, Z->nnz, cnt, trp, trow_tmp, tval_tmp, trow, tval, st));
        return FPS_OK;
    }

    // out = Z^p in (or (Z^T)^p in); in and out are distinct from t0/t1
    fps_status apply(const fps_csr_view* Z, int p, bool transpose, const double* in, double* out, hipStream_t st)
    {
        if (p == 0) {
            HIP_TRY(hipMemcpyAsync(out, in, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st));
            return FPS_OK;
        }
        const int64_t* rp = transpose ? trp : Z->row_ptr;
        const int32_t* cl = transpose ? trow : Z->col;
        const double* vl = transpose ? tval : Z->val;
        const double* cur = in;
        for (int i = 0; i < p; ++i) {
            double* dst = (i == p - 1) ? out : ((i % 2) ? t1 : t0);
            HIP_TRY(launch_spmv(rp, cl, vl, n, cur, dst, st));
            cur = dst;
        }
        return FPS_OK;
    }

    // The estimator on A = Z^p (the same steps as the block 1-norm estimator
    // of Higham and Tisseur with one column and itmax = 5).
    fps_status normest1(const fps_csr_view* Z, int p, double* est_out, int64_t* ind_out, int* iters, hipStream_t st)
    {
        const int itmax = 5;
        double* xv = x;
        double* yv = y;
        double* sv = s;
        double* sov = s_old;
        double* hv = zt;
        double* est_d = reinterpret_cast<double*>(small);
        unsigned int* flags = reinterpret_cast<unsigned int*>(small + 8);
        unsigned long long* res = reinterpret_cast<unsigned long long*>(small + 16);
        HIP_TRY(launch_fill_f64(xv, n, 1.0 / (double)n, st));
        double est = 0.0, est_old = 0.0;
        int64_t ind = -1, ind_best = -1;
        int k = 0;
        for (k = 1;; ++k) {
            FPS_TRY(apply(Z, p, false, xv, yv, st));
            HIP_TRY(launch_abs_sum_ordered(yv, n, est_d, st));
            HIP_TRY(hipMemcpyAsync(&est, est_d, sizeof(double), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (est > est_old || k == 2) ind_best = ind;
            if (k >= 2 && est <= est_old) {
                est = est_old;
                break;
            }
            est_old = est;
            if (k > itmax) break;
            // both flags set (two 32-bit ones) by a fill kernel, no host copy
            HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(flags), 1, 0x0000000100000001ull, st));
            HIP_TRY(launch_sign(yv, n, sov, k >= 2 ? 1 : 0, sv, flags, st));
            if (k >= 2) {  // the new sign vector parallel to the previous one
                unsigned int f[2] = {0u, 0u};
                HIP_TRY(hipMemcpyAsync(f, flags, sizeof(f), hipMemcpyDeviceToHost, st));
                HIP_TRY(hipStreamSynchronize(st));
                if (f[0] || f[1]) break;
            }
            std::swap(sv, sov);  // sov: the current sign vector
            FPS_TRY(apply(Z, p, true, sov, hv, st));
            HIP_TRY(launch_fill_u64(res, 1, 0ull, st));
            HIP_TRY(launch_fill_u64(res + 1, 1, ~0ull, st));
            HIP_TRY(launch_absmax(hv, n, res, st));
            unsigned long long r[2] = {0ull, 0ull};
            double hbest = 0.0;
            HIP_TRY(hipMemcpyAsync(r, res, sizeof(r), hipMemcpyDeviceToHost, st));
            if (k >= 2) HIP_TRY(hipMemcpyAsync(&hbest, hv + ind_best, sizeof(double), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            double hmax = 0.0;
            std::memcpy(&hmax, &r[0], sizeof(double));
            if (k >= 2 && hmax == std::fabs(hbest)) break;
            ind = (int64_t)r[1];
            HIP_TRY(launch_unit_vector(xv, n, ind, st));
        }
        *est_out = est;
        if (ind_out) *ind_out = ind_best;
        if (iters) *iters = k;
        return FPS_OK;
    }
};

// Eq. 37: z[0] = 1, z[i] estimates for 1 <= i <= K, alpha^i beyond (Lemma 1).
fps_status power_norm_bounds(EstWork& w, const fps_csr_view* Z, int K, int tmax, double* z, hipStream_t st)
{
    z[0] = 1.0;
    const int top = std::min(tmax, K);
    for (int i = 1; i <= top; ++i) FPS_TRY(w.normest1(Z, i, &z[i], nullptr, nullptr, st));
    if (tmax > K) {
        double alpha = 0.0;
        for (int k = (K + 1) / 2; k <= K; ++k) {
            const double r = std::pow(z[k], 1.0 / (double)k);
            if (r > alpha) alpha = r;
        }
        for (int i = K + 1; i <= tmax; ++i) z[i] = std::pow(alpha, (double)i);
    }
    return FPS_OK;
}

// Eq. 34 and Algorithm 2 step 3: N, q and the tail T_N.
fps_status series_degree(const double* a, int L, const double* z, double eps_tol, int* N_out, int* q_out,
                         double* tail)
{
    std::vector<double> T((size_t)L + 1);
    T[(size_t)L] = 0.0;
    for (int m = L - 1; m >= 0; --m) T[(size_t)m] = T[(size_t)m + 1] + std::fabs(a[m]) * z[m];
    int N = L;
    for (int m = 1; m <= L; ++m)
        if (T[(size_t)m] <= 0.5 * eps_tol) {
            N = m;
            break;
        }
    if (N >= L)
        return set_error(FPS_ERR_INVALID_ARG, "the %d coefficients given do not reach the tolerance (eq. 34 needs more)", L);
    int q = 0;
    while ((int64_t)(q + 1) * (q + 1) <= (int64_t)(N - 1)) ++q;
    if (q < 1) q = 1;
    *N_out = N;
    *q_out = q;
    *tail = T[(size_t)N];
    return FPS_OK;
}

// View of a canonical CSR for the kernels, with its row summaries and
// structure words.
MatView canon_view(const fps_csr_view* v, const RowInfo* info, const uint2* sw, const int32_t* nw)
{
    return MatView{v->row_ptr, v->row_ptr + 1, v->col, v->val, info, sw, nw};
}

}  // namespace

// ===========================================================================
// Plan
// ===========================================================================

struct fps_plan_s {
    MemAcct acct;  // first member: it outlives every buffer of the plan
    fps_csr_view Z{};
    std::vector<double> c;
    int m = 0, s = 0;
    double tau = 0.0;
    // per-row thresholds (device, n) of a batch group: row r drops |x| < tau_row[r]
    const double* tau_row = nullptr;
    // per-row multiply-add counters (device, n) added to by every stage's analysis
    int64_t* prod_acc = nullptr;
    // adaptive filter
    bool adaptive = false;
    double eps = 0.0, e_r = 0.0;
    int max_alg1 = 200;
    int alg1_dev_iters = 0;  // Algorithm 1 iterations on the device: 0 learned, < 0 host-driven
    std::vector<double> znorm, zeta, sigma;
    uint64_t flags = 0;
    // series mode (fps_plan_create_series)
    bool series = false;
    int series_N = 0, series_q = 0;
    double series_tail = 0.0, series_budget = 0.0;
    std::vector<double> series_z;
    Schedule sc;
    Engine eng;
    std::vector<std::unique_ptr<SlackMatrix>> P;  // P[j], j >= 2
    SlackMatrix S[2];
    CanonMatrix result;
    const SlackMatrix* final_m = nullptr;
    std::vector<StageRecord> rec;
    std::vector<hipEvent_t> ring;  // [slot][stage][2] when timing
    int n_stages = 0;
    hipStream_t last_stream = nullptr;
    int64_t evals = 0;
    // FPS_FLAG_TIMING: evaluations sampled so far, and the sample and
    // evaluation counts at the last statistics query
    int64_t timed = 0, timed_seen = 0, evals_seen = 0;
    bool timing_now = false;  // the evaluation being enqueued records events
    int64_t resizes = 0;
    bool evaluated = false;
    bool sized_once = false;

    int stage_count() const
    {
        // powers + the first Horner state + the Horner steps
        return (sc.J > 1 ? sc.J - 1 : 0) + sc.b + 2;
    }

    // Terms of block i over series indices i*q + j, j = 0..jmax (eq. 13).
    void block_terms(int i, int jmax, Terms* T, const MatView& zv) const
    {
        T->n = 0;
        for (int j = 0; j <= jmax; ++j) {
            const int k = i * sc.q + j;
            if (k > m) break;
            if (c[(size_t)k] == 0.0) continue;
            const int t = T->n++;
            T->coef[t] = c[(size_t)k];
            if (j == 0) {
                T->beg[t] = nullptr;
                T->end[t] = nullptr;
                T->col[t] = nullptr;
                T->val[t] = nullptr;
                T->info[t] = nullptr;
                T->sw[t] = nullptr;
                T->nw[t] = nullptr;
            } else {
                const MatView v = (j == 1) ? zv : P[(size_t)j]->view();
                T->beg[t] = v.beg;
                T->end[t] = v.end;
                T->col[t] = v.col;
                T->val[t] = v.val;
                T->info[t] = v.info;
                T->sw[t] = v.sw;
                T->nw[t] = v.nw;
            }
        }
    }

    // Matrix terms of block `block` (eq. 13) for the byte accounting: -1 = Z,
    // otherwise the stage that produced P_j.
    void add_term_sources(StageRecord* r, int block, int jmax, const std::vector<int>& pow_stage) const
    {
        for (int j = 1; j <= jmax; ++j) {
            const int kk = block * sc.q + j;
            if (kk > m) break;
            if (c[(size_t)kk] == 0.0) continue;
            r->term_src.push_back(j == 1 ? -1 : pow_stage[(size_t)j]);
        }
    }

    fps_status run_eval(hipStream_t s, bool size, bool host_alg1 = false)
    {
        const int64_t n = Z.n;
        n_stages = 0;
        eng.eval_id++;
        HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(eng.ws.counters.p),
                                (int64_t)(sizeof(StageCounters) / 8) * eng.ws.max_stages, 0ull, s));
        RowInfo* zinfo = eng.ws.zinfo.as<RowInfo>();
        FPS_TRY(eng.ws.zsw.ensure(sizeof(uint2) * (size_t)std::max<int64_t>(Z.nnz, 1)));
        uint2* zsw = eng.ws.zsw.as<uint2>();
        int32_t* znw = eng.ws.znw.as<int32_t>();
        HIP_TRY(launch_rowinfo_csr(Z.row_ptr, Z.col, Z.val, n, zinfo, zsw, znw, s));
        const MatView zv = canon_view(&Z, zinfo, zsw, znw);
        // dropped-entry statistics (fixed threshold): every stage's removed
        // entries are computed, so the row skip is off
        const bool dstats = (flags & FPS_FLAG_DROP_STATS) && !adaptive && tau > 0.0;
        const double skip_tau = (flags & FPS_FLAG_NO_SKIP) || dstats || tau <= 0.0 ? 0.0 : tau * (1.0 - 1e-6);
        // a batch group: per-row thresholds, the same 1e-6 margin for the skip
        const double* tau_rows = adaptive ? nullptr : tau_row;
        const double skip_rel = (flags & FPS_FLAG_NO_SKIP) ? 0.0 : 1.0 - 1e-6;
        unsigned long long* dsum = nullptr;
        if (dstats) {
            FPS_TRY(eng.ws.dsum.ensure(sizeof(unsigned long long) * (size_t)std::max<int64_t>(n, 1)));
            dsum = eng.ws.dsum.as<unsigned long long>();
            HIP_TRY(launch_fill_u64(dsum, n, 0ull, s));
        }
        // after a filtered product: the largest column sum, then the sums cleared
        auto drop_stats = [&](StageArgs& a) {
            a.dsum = dsum;
            a.dscale = dstats ? std::ldexp(1.0, 40) / tau : 0.0;
            a.dthr = 0.0;
            a.dcount = 1;
        };
        auto drop_norm = [&](int idx) -> fps_status {
            if (!dstats) return FPS_OK;
            HIP_TRY(launch_max_u64(dsum, n, &eng.ctr(idx)->dropped_colmax, s));
            HIP_TRY(launch_fill_u64(dsum, n, 0ull, s));
            return FPS_OK;
        };

        const int nst = stage_count();
        const size_t slot = (size_t)(timed % kTimingRing);
        auto begin_stage = [&](Kind k, int index) -> StageRecord* {
            StageRecord* r = &rec[(size_t)n_stages];
            r->kind = (int)k;
            r->index = index;
            r->a_src = r->b_src = r->e_src = -1;
            r->a_is_z = r->b_is_z = false;
            r->term_src.clear();
            r->eps_g = r->threshold = r->dropped = 0.0;
            r->alg1_iters = 0;
            r->alg1_device = false;
            r->alg1_mode = 0;
            r->wide_rows = false;
            r->small = false;
            r->dense = 0;
            r->ev0 = r->ev1 = nullptr;
            if (timing_now) {
                r->ev0 = ring[(slot * (size_t)nst + (size_t)n_stages) * 2];
                r->ev1 = ring[(slot * (size_t)nst + (size_t)n_stages) * 2 + 1];
            }
            return r;
        };

        std::vector<int> pow_stage((size_t)sc.J + 2, -1);
        // step 1: filtered powers P_{j+1} = D_tau(Z (x) P_j)   (eq. 11)
        for (int j = 1; j + 1 <= sc.J; ++j) {
            StageArgs a{};
            a.prod_acc = prod_acc;
            a.mode = kModeProduct;
            a.tau = adaptive ? 0.0 : tau;
            a.skip_tau = adaptive ? 0.0 : skip_tau;
            a.tau_row = tau_rows;
            a.skip_rel = skip_rel;
            a.A = zv;
            a.B = (j == 1) ? zv : P[(size_t)j]->view();
            a.has_e = 0;
            drop_stats(a);
            if (adaptive)
                FPS_TRY(eng.alg1_fuse(n_stages, zeta[(size_t)j + 1], host_alg1 ? -1 : alg1_dev_iters, a, s));
            StageRecord* r = begin_stage(Kind::Power, j + 1);
            r->a_is_z = true;
            r->b_is_z = (j == 1);
            r->b_src = (j == 1) ? -1 : pow_stage[(size_t)j];
            FPS_TRY(eng.run(n_stages, a, *P[(size_t)j + 1], s, size, r));
            FPS_TRY(drop_norm(n_stages));
            if (adaptive)
                FPS_TRY(eng.alg1(n_stages, *P[(size_t)j + 1], zeta[(size_t)j + 1], e_r, max_alg1, s, r,
                                 host_alg1 ? -1 : alg1_dev_iters));
            pow_stage[(size_t)j + 1] = n_stages++;
        }

        auto run_sum = [&](Kind k, int index, int block, int jmax, SlackMatrix& out) -> fps_status {
            StageArgs a{};
            a.prod_acc = prod_acc;
            a.mode = kModeSum;
            a.tau = 0.0;
            a.skip_tau = 0.0;
            block_terms(block, jmax, &a.T, zv);
            a.has_e = 0;
            StageRecord* r = begin_stage(k, index);
            add_term_sources(r, block, jmax, pow_stage);
            FPS_TRY(eng.run(n_stages, a, out, s, size, r));
            n_stages++;
            return FPS_OK;
        };

        if (sc.b == 1) {
            FPS_TRY(run_sum(Kind::Block, 0, 0, sc.q - 1, S[0]));
            final_m = &S[0];
        } else {
            int cur = 0;
            if (sc.g) {
                FPS_TRY(run_sum(Kind::GStep, 1, sc.b - 2, sc.q, S[cur]));  // eq. 14, g = 1
            } else {
                FPS_TRY(run_sum(Kind::Block, sc.b - 1, sc.b - 1, sc.q - 1, S[cur]));
            }
            int s_stage = n_stages - 1;
            for (int i = sc.start; i <= sc.b - 1; ++i) {
                // S_i = D_tau(Bhat_{b-1-i} + P_q (x) S_{i-1}) with the block summed inside the step
                StageArgs a{};
                a.prod_acc = prod_acc;
                a.mode = kModeProduct;
                a.tau = adaptive ? 0.0 : tau;
                a.skip_tau = adaptive ? 0.0 : skip_tau;
                a.tau_row = tau_rows;
                a.skip_rel = skip_rel;
                a.A = (sc.q == 1) ? zv : P[(size_t)sc.q]->view();
                a.B = S[cur].view();
                a.has_e = 0;
                block_terms(sc.b - 1 - i, sc.q - 1, &a.T, zv);
                a.has_blk = a.T.n > 0 ? 1 : 0;
                drop_stats(a);
                if (adaptive)
                    FPS_TRY(eng.alg1_fuse(n_stages, sigma[(size_t)i], host_alg1 ? -1 : alg1_dev_iters, a, s));
                StageRecord* r = begin_stage(Kind::Horner, i);
                r->a_is_z = (sc.q == 1);
                r->a_src = (sc.q == 1) ? -1 : pow_stage[(size_t)sc.q];
                r->b_src = s_stage;
                add_term_sources(r, sc.b - 1 - i, sc.q - 1, pow_stage);
                FPS_TRY(eng.run(n_stages, a, S[1 - cur], s, size, r));
                FPS_TRY(drop_norm(n_stages));
                if (adaptive)
                    FPS_TRY(eng.alg1(n_stages, S[1 - cur], sigma[(size_t)i], e_r, max_alg1, s, r,
                                     host_alg1 ? -1 : alg1_dev_iters));
                s_stage = n_stages++;
                cur = 1 - cur;
            }
            final_m = &S[cur];
        }
        FPS_TRY(eng.compact(*final_m, result, s));
        if (size) FPS_TRY(eng.grow_for_strides(s));
        return FPS_OK;
    }
};

extern "C" {

int32_t fps_abi_version(void) { return FPS_ABI_VERSION; }

const char* fps_status_string(fps_status s)
{
    switch (s) {
    case FPS_OK: return "ok";
    case FPS_ERR_INVALID_ARG: return "invalid argument";
    case FPS_ERR_BAD_CSR: return "bad CSR input";
    case FPS_ERR_OUT_OF_MEMORY: return "out of device memory";
    case FPS_ERR_HIP: return "HIP error";
    case FPS_ERR_CAPACITY: return "capacity exceeded";
    case FPS_ERR_NOT_READY: return "not ready";
    default: return "unknown status";
    }
}

const char* fps_last_error(void) { return g_last_error.c_str(); }

fps_status fps_schedule(int32_t m, int32_t s, int32_t* N, int32_t* q, int32_t* b, int32_t* g, int32_t* J,
                        int32_t* start, int32_t* n_spgemm)
{
    Schedule sc;
    if (!make_schedule(m, s, &sc)) return set_error(FPS_ERR_INVALID_ARG, "need m >= 0 and s >= 1");
    if (N) *N = sc.N;
    if (q) *q = sc.q;
    if (b) *b = sc.b;
    if (g) *g = sc.g;
    if (J) *J = sc.J;
    if (start) *start = sc.start;
    if (n_spgemm) *n_spgemm = sc.nsp;
    return FPS_OK;
}

}  // extern "C"

// fps_plan_create_ex with a limit on the device bytes the plan may hold
// (creation and every later evaluation); past it an allocation fails with
// FPS_ERR_CAPACITY.
static fps_status plan_create_limited(fps_plan* out, const fps_csr_view* Z, const double* coeffs, int32_t m, int32_t s,
                                      const fps_filter_opts* opts, uint64_t flags, fps_stream stream, size_t mem_cap,
                                      bool (*extend)(void*, MemAcct*, size_t) = nullptr, void* extend_ctx = nullptr);

extern "C" {

fps_status fps_plan_create_ex(fps_plan* out, const fps_csr_view* Z, const double* coeffs, int32_t m, int32_t s,
                              const fps_filter_opts* opts, uint64_t flags, fps_stream stream)
{
    return plan_create_limited(out, Z, coeffs, m, s, opts, flags, stream, SIZE_MAX);
}

}  // extern "C"

static fps_status plan_create_limited(fps_plan* out, const fps_csr_view* Z, const double* coeffs, int32_t m, int32_t s,
                                      const fps_filter_opts* opts, uint64_t flags, fps_stream stream, size_t mem_cap,
                                      bool (*extend)(void*, MemAcct*, size_t), void* extend_ctx)
{
    g_last_error.clear();
    if (!out) return set_error(FPS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!opts) return set_error(FPS_ERR_INVALID_ARG, "opts is NULL");
    FPS_TRY(check_view(Z, "Z", -1));
    if (!coeffs) return set_error(FPS_ERR_INVALID_ARG, "coeffs is NULL");
    if (m < 0) return set_error(FPS_ERR_INVALID_ARG, "m must be >= 0");
    if (s < 1 || s > FPS_MAX_S) return set_error(FPS_ERR_INVALID_ARG, "s must be in [1, %d]", FPS_MAX_S);
    for (int k = 0; k <= m; ++k)
        if (!std::isfinite(coeffs[k])) return set_error(FPS_ERR_INVALID_ARG, "coefficient %d is not finite", k);
    Schedule sc;
    make_schedule(m, s, &sc);
    const bool adaptive = opts->filter == FPS_FILTER_ADAPTIVE;
    if (opts->filter == FPS_FILTER_FIXED) {
        if (!std::isfinite(opts->tau) || opts->tau < 0.0)
            return set_error(FPS_ERR_INVALID_ARG, "tau must be finite and >= 0");
    } else if (adaptive) {
        if (!std::isfinite(opts->eps) || !(opts->eps > 0.0))
            return set_error(FPS_ERR_INVALID_ARG, "eps must be finite and > 0");
        if (!std::isfinite(opts->e_r) || opts->e_r < 0.0)
            return set_error(FPS_ERR_INVALID_ARG, "e_r must be finite and >= 0");
        if (opts->max_alg1_iters < 0) return set_error(FPS_ERR_INVALID_ARG, "max_alg1_iters must be >= 0");
        if (opts->alg1_device_iters < -1 || opts->alg1_device_iters > 64)
            return set_error(FPS_ERR_INVALID_ARG, "alg1_device_iters must be in [-1, 64]");
    } else {
        return set_error(FPS_ERR_INVALID_ARG, "unknown filter %d", opts->filter);
    }
    // The integer column sums of Algorithm 1 and of the dropped-entry
    // statistics add at most 2^40 + 1 per entry into 64 bits: exact while a
    // column holds fewer than 2^24 entries, which n < 2^24 guarantees.
    if ((adaptive || (flags & FPS_FLAG_DROP_STATS)) && Z->n >= kColSumMaxN)
        return set_error(FPS_ERR_CAPACITY, "n = %lld: Algorithm 1 and FPS_FLAG_DROP_STATS need n < 2^24",
                         (long long)Z->n);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!(flags & FPS_FLAG_NO_VALIDATE)) FPS_TRY(validate_on_device(Z, "Z", st));

    std::unique_ptr<fps_plan_s> p(new (std::nothrow) fps_plan_s());
    if (!p) return set_error(FPS_ERR_OUT_OF_MEMORY, "host allocation failed");
    p->acct.cap = mem_cap;
    p->acct.extend = extend;
    p->acct.ctx = extend_ctx;
    AcctScope scope(&p->acct);
    p->Z = *Z;
    p->c.assign(coeffs, coeffs + m + 1);
    p->m = m;
    p->s = s;
    p->tau = adaptive ? 0.0 : opts->tau;
    p->flags = flags;
    p->sc = sc;
    p->adaptive = adaptive;
    if (adaptive) {
        p->eps = opts->eps;
        p->e_r = opts->e_r;
        p->max_alg1 = opts->max_alg1_iters > 0 ? opts->max_alg1_iters : 200;
        p->alg1_dev_iters = opts->alg1_device_iters;
        const int tmax = std::max(sc.q, sc.q * (sc.b - 1));
        if (opts->znorm) {
            p->znorm.assign(opts->znorm, opts->znorm + tmax + 1);
        } else {  // the bounds of eq. 37 from the 1-norm estimator
            p->znorm.assign((size_t)tmax + 1, 0.0);
            EstWork w;
            FPS_TRY(w.init(Z, st));
            FPS_TRY(power_norm_bounds(w, Z, 10, tmax, p->znorm.data(), st));
        }
        for (double v : p->znorm)
            if (!std::isfinite(v) || v < 0.0) return set_error(FPS_ERR_INVALID_ARG, "znorm values must be finite and >= 0");
        fnt_thresholds(p->c, m, sc, p->eps, p->znorm, p->zeta, p->sigma);
    }
    const int stages = p->stage_count();
    if (stages > FPS_MAX_STAGES)
        return set_error(FPS_ERR_CAPACITY, "schedule needs %d stages, at most %d supported", stages, FPS_MAX_STAGES);
    FPS_TRY(p->eng.init(Z->n, stages, flags, st));
    p->P.resize((size_t)std::max(p->sc.J, 1) + 2);
    for (auto& x : p->P) x.reset(new SlackMatrix());
    p->rec.assign((size_t)stages, StageRecord{});
    if (flags & FPS_FLAG_TIMING) {
        p->ring.assign((size_t)kTimingRing * (size_t)stages * 2, nullptr);
        // timestamps only: no system-scope fence (which would flush caches at every record)
        for (auto& e : p->ring) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    *out = p.release();
    return FPS_OK;
}

extern "C" {

fps_status fps_plan_create(fps_plan* out, const fps_csr_view* Z, const double* coeffs, int32_t m, int32_t s,
                           double tau, uint64_t flags, fps_stream stream)
{
    fps_filter_opts o{};
    o.filter = FPS_FILTER_FIXED;
    o.tau = tau;
    return fps_plan_create_ex(out, Z, coeffs, m, s, &o, flags, stream);
}

fps_status fps_eval(fps_plan p, fps_stream stream)
{
    if (!p) return set_error(FPS_ERR_INVALID_ARG, "plan is NULL");
    AcctScope scope(&p->acct);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool size = (p->flags & FPS_FLAG_SYNC_SIZES) || !p->sized_once;
    p->last_stream = s;
    // sampled: the first evaluation after a statistics query, then every 8th
    p->timing_now = !p->ring.empty() && ((p->evals - p->evals_seen) % kTimingEvery == 0);
    fps_status st = p->run_eval(s, size);
    if (st != FPS_OK) return st;
    if (size) p->sized_once = true;
    if (p->timing_now) p->timed++;
    p->evals++;
    p->evaluated = true;
    return FPS_OK;
}

static fps_status read_errors(fps_plan p, unsigned long long* err)
{
    std::vector<StageCounters> c((size_t)p->n_stages);
    if (p->n_stages > 0)
        HIP_TRY(hipMemcpy(c.data(), p->eng.ws.counters.p, sizeof(StageCounters) * (size_t)p->n_stages,
                          hipMemcpyDeviceToHost));
    unsigned long long e = 0;
    for (auto& x : c) e |= x.errors;
    *err = e;
    return FPS_OK;
}

// Synchronises, checks the device error flags and re-runs with sizing if a
// learned capacity turned out too small.
static fps_status finish(fps_plan p)
{
    AcctScope scope(&p->acct);
    HIP_TRY(hipStreamSynchronize(p->last_stream));
    unsigned long long err = 0;
    FPS_TRY(read_errors(p, &err));
    if (err & kErrColumnOutsideWindow) return set_error(FPS_ERR_HIP, "internal error: column outside its row window");
    if (err & (kErrCapacity | kErrNeedsGlobal | kErrAlg1Pending)) {
        // re-run with sizing (and, if Algorithm 1 needed more iterations than
        // were launched on the device, with the host-driven loop)
        p->resizes++;
        p->timing_now = false;
        FPS_TRY(p->run_eval(p->last_stream, true, (err & kErrAlg1Pending) != 0));
        HIP_TRY(hipStreamSynchronize(p->last_stream));
        FPS_TRY(read_errors(p, &err));
        if (err) return set_error(FPS_ERR_CAPACITY, "stage workspace exceeded after re-sizing (flags %llx)", err);
    }
    return FPS_OK;
}

fps_status fps_result_nnz(fps_plan p, int64_t* nnz)
{
    if (!p || !nnz) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    if (!p->evaluated) return set_error(FPS_ERR_NOT_READY, "no evaluation has run on this plan");
    FPS_TRY(finish(p));
    HIP_TRY(hipMemcpy(nnz, p->result.rp.as<int64_t>() + p->Z.n, sizeof(int64_t), hipMemcpyDeviceToHost));
    return FPS_OK;
}

fps_status fps_result_copy(fps_plan p, int64_t* row_ptr, int32_t* col, double* val, fps_stream stream)
{
    if (!p || !row_ptr) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    if (!p->evaluated) return set_error(FPS_ERR_NOT_READY, "no evaluation has run on this plan");
    int64_t nnz = 0;
    FPS_TRY(fps_result_nnz(p, &nnz));
    if (nnz > 0 && (!col || !val)) return set_error(FPS_ERR_INVALID_ARG, "null col/val with nnz > 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = p->Z.n;
    HIP_TRY(hipMemcpyAsync(row_ptr, p->result.rp.p, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz > 0) {
        HIP_TRY(hipMemcpyAsync(col, p->result.col.p, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(val, p->result.val.p, sizeof(double) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
    }
    return FPS_OK;
}

fps_status fps_get_stats(fps_plan p, fps_stats* st)
{
    if (!p || !st) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    std::memset(st, 0, sizeof(*st));
    st->N = p->sc.N;
    st->q = p->sc.q;
    st->b = p->sc.b;
    st->g = p->sc.g;
    st->J = p->sc.J;
    st->start = p->sc.start;
    st->n_spgemm = p->sc.nsp;
    st->evals = p->evals;
    st->resizes = p->resizes;
    if (!p->evaluated) return FPS_OK;
    FPS_TRY(finish(p));
    const int ns = p->n_stages;
    std::vector<StageCounters> c((size_t)ns);
    HIP_TRY(hipMemcpy(c.data(), p->eng.ws.counters.p, sizeof(StageCounters) * (size_t)ns, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&st->nnz_out, p->result.rp.as<int64_t>() + p->Z.n, sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<Alg1State> a1((size_t)ns * 3);
    if (p->adaptive && ns > 0)
        HIP_TRY(hipMemcpy(a1.data(), p->eng.alg1st.p, sizeof(Alg1State) * 3 * (size_t)ns, hipMemcpyDeviceToHost));
    std::vector<std::array<unsigned long long, kPartCount>> tot((size_t)ns);
    for (int i = 0; i < ns; ++i) {
        const int kind = p->rec[(size_t)i].kind;
        const int32_t mode = (kind == FPS_STAGE_POWER || kind == FPS_STAGE_HORNER) ? kModeProduct : kModeSum;
        FPS_TRY(p->eng.stage_totals(i, mode, tot[(size_t)i].data()));
    }
    st->n_stages = std::min(ns, FPS_MAX_STAGES);
    const double n1 = (double)(p->Z.n + 1);
    double bytes = 0.0, ms_total = 0.0;
    int launches = 0;
    auto kept = [&](int i) { return (double)tot[(size_t)i][kPartKept]; };
    for (int i = 0; i < ns && i < FPS_MAX_STAGES; ++i) {
        const StageRecord& r = p->rec[(size_t)i];
        st->kind[i] = r.kind;
        st->index[i] = r.index;
        st->stage_products[i] = (int64_t)tot[(size_t)i][kPartProducts];
        st->stage_eps_g[i] = r.eps_g;
        st->stage_threshold[i] = r.threshold;
        st->stage_dropped[i] = r.dropped;
        st->stage_alg1_iters[i] = r.alg1_iters;
        st->stage_alg1_mode[i] = r.alg1_mode;
        st->stage_dense[i] = r.dense;
        st->stage_small[i] = r.small ? 1 : 0;
        st->stage_max_ns[i] = p->eng.learned_ns[(size_t)i];
        st->stage_max_words[i] = p->eng.learned_words[(size_t)i];
        if (r.dense) st->dense_ld = p->eng.d_ld;
        st->stage_rows_skipped[i] = (int64_t)tot[(size_t)i][kPartRowsSkipped];
        if (r.alg1_device) {
            const Alg1State& f = a1[(size_t)i * 3 + 2];
            st->stage_threshold[i] = f.t;
            st->stage_dropped[i] = f.c;
            st->stage_alg1_iters[i] = f.it;
        }
        if ((p->flags & FPS_FLAG_DROP_STATS) && !p->adaptive && p->tau > 0.0 &&
            (r.kind == FPS_STAGE_POWER || r.kind == FPS_STAGE_HORNER)) {
            const StageCounters& k = c[(size_t)i];
            st->stage_n_dropped[i] = (int64_t)k.n_dropped;
            double mx;
            std::memcpy(&mx, &k.dropped_max, sizeof(mx));
            st->stage_dropped_max[i] = mx;
            st->stage_dropped[i] = std::ldexp((double)k.dropped_colmax, -40) * p->tau;
        }
        st->stage_nnz[i] = (int64_t)tot[(size_t)i][kPartKept];
        st->products += (int64_t)tot[(size_t)i][kPartProducts];
        st->products_skipped += (int64_t)tot[(size_t)i][kPartProductsSkipped];
        st->rows_skipped += (int64_t)tot[(size_t)i][kPartRowsSkipped];
        st->rows_global += (int64_t)c[(size_t)i].fb2_count;
        st->rows_wide += r.wide_rows ? p->Z.n - (int64_t)c[(size_t)i].fb2_count : (int64_t)c[(size_t)i].rows_wide;
        const double za = (double)p->Z.nnz;
        double sb = 0.0;
        if (r.kind == FPS_STAGE_POWER || r.kind == FPS_STAGE_HORNER) {
            const double na = r.a_is_z ? za : (r.a_src >= 0 ? kept(r.a_src) : 0.0);
            const double nb = r.b_is_z ? za : (r.b_src >= 0 ? kept(r.b_src) : 0.0);
            const double ne = r.e_src >= 0 ? kept(r.e_src) : 0.0;
            double nt = 0.0;  // fused block terms
            for (int src : r.term_src) nt += (src < 0) ? za : kept(src);
            const double skipped = (double)tot[(size_t)i][kPartRowsSkipped];
            const double n0 = (double)p->Z.n;
            if (n0 > 0.0 && skipped >= n0) {
                // every row proven empty: the analysis reads the left operand,
                // the 16-byte summary of each referenced row and of each block
                // term's row, nothing else
                sb = 12.0 * na + 16.0 * na + 16.0 * n0 * (double)r.term_src.size() + 8.0 * n1;
            } else {
                const double f = n0 > 0.0 ? (n0 - skipped) / n0 : 1.0;
                const double operands = 3.0 + (r.e_src >= 0 ? 1.0 : 0.0) + (double)r.term_src.size();
                sb = 12.0 * (na + f * (nb + ne + nt) + kept(i)) + 8.0 * n1 * operands;
            }
        } else {
            // coefficient sum: every stored term matrix read once, the sum written once
            double in = 0.0;
            for (int src : r.term_src) in += (src < 0) ? za : kept(src);
            sb = 12.0 * (in + kept(i)) + 8.0 * n1 * (double)(r.term_src.size() + 1);
        }
        st->stage_bytes[i] = sb;
        bytes += sb;
        if (!p->ring.empty()) {
            // average over the sampled evaluations since the last query (the
            // latest sampled one if none)
            const int64_t fresh = p->timed - p->timed_seen;
            const int64_t held = fresh > 0 ? std::min<int64_t>(fresh, kTimingRing) : std::min<int64_t>(p->timed, 1);
            const size_t nst = (size_t)p->stage_count();
            double sum = 0.0;
            for (int64_t e = p->timed - held; e < p->timed; ++e) {
                const size_t slot = (size_t)(e % kTimingRing);
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, p->ring[(slot * nst + (size_t)i) * 2],
                                            p->ring[(slot * nst + (size_t)i) * 2 + 1]));
                sum += ms;
            }
            const double avg = held > 0 ? sum / (double)held : 0.0;
            st->stage_ms[i] = avg;
            ms_total += avg;
            launches++;
        }
    }
    st->bytes_algorithmic = bytes;
    st->numeric_ms = ms_total;
    st->numeric_launches = launches;
    p->timed_seen = p->timed;
    p->evals_seen = p->evals;
    return FPS_OK;
}

void fps_plan_destroy(fps_plan p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->last_stream);
    for (auto& e : p->ring)
        if (e) (void)hipEventDestroy(e);
    delete p;
}

// ===========================================================================
// Single stages
// ===========================================================================

struct fps_matrix_s {
    CanonMatrix m;
    int64_t nnz = 0;
};

static fps_status finish_single(Engine& eng, SlackMatrix& out, hipStream_t s, fps_matrix* res)
{
    std::unique_ptr<fps_matrix_s> mm(new (std::nothrow) fps_matrix_s());
    if (!mm) return set_error(FPS_ERR_OUT_OF_MEMORY, "host allocation failed");
    FPS_TRY(eng.compact(out, mm->m, s));
    StageCounters c{};
    HIP_TRY(hipMemcpyAsync(&c, eng.ctr(0), sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&mm->nnz, mm->m.rp.as<int64_t>() + out.n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c.errors) return set_error(FPS_ERR_CAPACITY, "stage failed (device flags %llx)", c.errors);
    *res = mm.release();
    return FPS_OK;
}

fps_status fps_spgemm(fps_matrix* out, const fps_csr_view* A, const fps_csr_view* B, const fps_csr_view* E,
                      double tau, fps_stream stream)
{
    g_last_error.clear();
    if (!out) return set_error(FPS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    FPS_TRY(check_view(A, "A", -1));
    FPS_TRY(check_view(B, "B", A->n));
    if (E) FPS_TRY(check_view(E, "E", A->n));
    if (!std::isfinite(tau) || tau < 0.0) return set_error(FPS_ERR_INVALID_ARG, "tau must be finite and >= 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    FPS_TRY(validate_on_device(A, "A", s));
    FPS_TRY(validate_on_device(B, "B", s));
    if (E) FPS_TRY(validate_on_device(E, "E", s));
    const int64_t n = A->n;
    Engine eng;
    FPS_TRY(eng.init(n, 1, 0, s));
    // row info and structure words of each operand
    const fps_csr_view* ops[3] = {A, B, E};
    DevBuf info[3], words[3];
    RowInfo* ri[3] = {};
    uint2* sw[3] = {};
    int32_t* nw[3] = {};
    const size_t per = (sizeof(RowInfo) + sizeof(int32_t)) * (size_t)n;
    for (int i = 0; i < 3; ++i) {
        if (!ops[i]) continue;
        FPS_TRY(info[i].ensure(per));
        FPS_TRY(words[i].ensure(sizeof(uint2) * (size_t)std::max<int64_t>(ops[i]->nnz, 1)));
        ri[i] = info[i].as<RowInfo>();
        nw[i] = reinterpret_cast<int32_t*>(static_cast<char*>(info[i].p) + sizeof(RowInfo) * (size_t)n);
        sw[i] = words[i].as<uint2>();
        HIP_TRY(launch_rowinfo_csr(ops[i]->row_ptr, ops[i]->col, ops[i]->val, n, ri[i], sw[i], nw[i], s));
    }
    HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(eng.ws.counters.p), sizeof(StageCounters) / 8, 0ull, s));
    StageArgs a{};
    a.mode = kModeProduct;
    a.tau = tau;
    a.skip_tau = tau > 0.0 ? tau * (1.0 - 1e-6) : 0.0;
    a.A = canon_view(A, ri[0], sw[0], nw[0]);
    a.B = canon_view(B, ri[1], sw[1], nw[1]);
    a.has_e = E ? 1 : 0;
    if (E) a.E = canon_view(E, ri[2], sw[2], nw[2]);
    SlackMatrix res;
    FPS_TRY(eng.run(0, a, res, s, true, nullptr));
    return finish_single(eng, res, s, out);
}

fps_status fps_axpy(fps_matrix* out, int64_t n, int32_t nterms, const double* coefs, const fps_csr_view* terms,
                    fps_stream stream)
{
    g_last_error.clear();
    if (!out) return set_error(FPS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > FPS_MAX_N) return set_error(FPS_ERR_INVALID_ARG, "n out of range");
    if (nterms < 1 || nterms > kMaxTerms) return set_error(FPS_ERR_INVALID_ARG, "nterms must be in [1, %d]", kMaxTerms);
    if (!coefs || !terms) return set_error(FPS_ERR_INVALID_ARG, "null coefs/terms");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (int t = 0; t < nterms; ++t) {
        if (!std::isfinite(coefs[t])) return set_error(FPS_ERR_INVALID_ARG, "coefficient %d not finite", t);
        if (terms[t].row_ptr) {
            FPS_TRY(check_view(&terms[t], "term", n));
            FPS_TRY(validate_on_device(&terms[t], "term", s));
        }
    }
    Engine eng;
    FPS_TRY(eng.init(n, 1, 0, s));
    DevBuf info;
    std::vector<DevBuf> words((size_t)nterms);
    // per term: row summaries (16-byte aligned blocks), then word counts
    const size_t per = ((sizeof(RowInfo) + sizeof(int32_t)) * (size_t)n + 255) / 256 * 256;
    FPS_TRY(info.ensure(per * (size_t)nterms));
    StageArgs a{};
    a.mode = kModeSum;
    a.tau = 0.0;
    a.skip_tau = 0.0;
    a.T.n = nterms;
    for (int t = 0; t < nterms; ++t) {
        a.T.coef[t] = coefs[t];
        if (!terms[t].row_ptr) {
            a.T.beg[t] = a.T.end[t] = nullptr;
            a.T.col[t] = nullptr;
            a.T.val[t] = nullptr;
            a.T.info[t] = nullptr;
            a.T.sw[t] = nullptr;
            a.T.nw[t] = nullptr;
            continue;
        }
        char* base = static_cast<char*>(info.p) + t * per;
        RowInfo* ri = reinterpret_cast<RowInfo*>(base);
        int32_t* nw = reinterpret_cast<int32_t*>(base + sizeof(RowInfo) * (size_t)n);
        FPS_TRY(words[(size_t)t].ensure(sizeof(uint2) * (size_t)std::max<int64_t>(terms[t].nnz, 1)));
        uint2* sw = words[(size_t)t].as<uint2>();
        HIP_TRY(launch_rowinfo_csr(terms[t].row_ptr, terms[t].col, terms[t].val, n, ri, sw, nw, s));
        a.T.beg[t] = terms[t].row_ptr;
        a.T.end[t] = terms[t].row_ptr + 1;
        a.T.col[t] = terms[t].col;
        a.T.val[t] = terms[t].val;
        a.T.info[t] = ri;
        a.T.sw[t] = sw;
        a.T.nw[t] = nw;
    }
    HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(eng.ws.counters.p), sizeof(StageCounters) / 8, 0ull, s));
    SlackMatrix res;
    FPS_TRY(eng.run(0, a, res, s, true, nullptr));
    return finish_single(eng, res, s, out);
}

fps_status fps_matrix_nnz(fps_matrix m, int64_t* nnz)
{
    if (!m || !nnz) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    *nnz = m->nnz;
    return FPS_OK;
}

fps_status fps_matrix_copy(fps_matrix m, int64_t* row_ptr, int32_t* col, double* val, fps_stream stream)
{
    if (!m || !row_ptr) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    if (m->nnz > 0 && (!col || !val)) return set_error(FPS_ERR_INVALID_ARG, "null col/val with nnz > 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(row_ptr, m->m.rp.p, sizeof(int64_t) * (size_t)(m->m.n + 1), hipMemcpyDeviceToDevice, s));
    if (m->nnz > 0) {
        HIP_TRY(hipMemcpyAsync(col, m->m.col.p, sizeof(int32_t) * (size_t)m->nnz, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(val, m->m.val.p, sizeof(double) * (size_t)m->nnz, hipMemcpyDeviceToDevice, s));
    }
    return FPS_OK;
}

void fps_matrix_destroy(fps_matrix m) { delete m; }

fps_status fps_normest1(const fps_csr_view* Z, int32_t p, double* est, int64_t* ind, int32_t* iters, uint64_t flags,
                        fps_stream stream)
{
    g_last_error.clear();
    if (!est) return set_error(FPS_ERR_INVALID_ARG, "est is NULL");
    if (p < 0) return set_error(FPS_ERR_INVALID_ARG, "p must be >= 0");
    FPS_TRY(check_view(Z, "Z", -1));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!(flags & FPS_FLAG_NO_VALIDATE)) FPS_TRY(validate_on_device(Z, "Z", st));
    EstWork w;
    FPS_TRY(w.init(Z, st));
    int it = 0;
    FPS_TRY(w.normest1(Z, p, est, ind, &it, st));
    if (iters) *iters = it;
    return FPS_OK;
}

}  // extern "C"

// ---- the estimator without allocation -----------------------------------------

// Workspace of fps_normest1_noalloc: the estimator's pieces for the largest
// accepted matrix, then the validation flag.  One copy per GPU, held until the
// process ends; every call on that GPU shares it.
constexpr size_t kNoAllocEstBytes = est_bytes(FPS_NOALLOC_MAX_N, FPS_NOALLOC_MAX_NNZ);
constexpr size_t kScratchBytes = kNoAllocEstBytes + 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device with that device current (the host-side name of the array is not a
// device address).
fps_status scratch_address(void** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(FPS_ERR_CAPACITY, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(FPS_ERR_HIP, "hipGetSymbolAddress gave a null address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FPS_OK;
}

}  // namespace

extern "C" {

fps_status fps_normest1_noalloc(const fps_csr_view* Z, int32_t p, double* est, int64_t* ind, int32_t* iters,
                                uint64_t flags, fps_stream stream)
{
    g_last_error.clear();
    if (!est) return set_error(FPS_ERR_INVALID_ARG, "est is NULL");
    if (p < 0) return set_error(FPS_ERR_INVALID_ARG, "p must be >= 0");
    FPS_TRY(check_view(Z, "Z", -1));
    if (Z->n > FPS_NOALLOC_MAX_N || Z->nnz > FPS_NOALLOC_MAX_NNZ)
        return set_error(FPS_ERR_CAPACITY, "fps_normest1_noalloc: n = %lld, nnz = %lld beyond its limits (n <= %d, nnz <= %d)",
                         (long long)Z->n, (long long)Z->nnz, FPS_NOALLOC_MAX_N, FPS_NOALLOC_MAX_NNZ);
    void* base = nullptr;
    FPS_TRY(scratch_address(&base));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!(flags & FPS_FLAG_NO_VALIDATE))
        FPS_TRY(validate_on_device(Z, "Z", st,
                                   reinterpret_cast<unsigned long long*>(static_cast<char*>(base) + kNoAllocEstBytes)));
    EstWork w;
    FPS_TRY(w.init_at(Z, base, st));
    int it = 0;
    FPS_TRY(w.normest1(Z, p, est, ind, &it, st));
    if (iters) *iters = it;
    return FPS_OK;
}

fps_status fps_power_norm_bounds(const fps_csr_view* Z, int32_t K, int32_t tmax, double* z, uint64_t flags,
                                 fps_stream stream)
{
    g_last_error.clear();
    if (!z) return set_error(FPS_ERR_INVALID_ARG, "z is NULL");
    if (K < 2 || (K % 2) != 0) return set_error(FPS_ERR_INVALID_ARG, "K must be even and >= 2");
    if (tmax < 0) return set_error(FPS_ERR_INVALID_ARG, "tmax must be >= 0");
    FPS_TRY(check_view(Z, "Z", -1));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!(flags & FPS_FLAG_NO_VALIDATE)) FPS_TRY(validate_on_device(Z, "Z", st));
    EstWork w;
    FPS_TRY(w.init(Z, st));
    return power_norm_bounds(w, Z, K, tmax, z, st);
}

fps_status fps_plan_create_series(fps_plan* out, const fps_csr_view* Z, const double* a, int32_t L,
                                  const fps_series_opts* opts, uint64_t flags, fps_stream stream)
{
    g_last_error.clear();
    if (!out) return set_error(FPS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!opts || !a) return set_error(FPS_ERR_INVALID_ARG, "null a/opts");
    if (L < 2) return set_error(FPS_ERR_INVALID_ARG, "L must be >= 2");
    if (!std::isfinite(opts->eps_tol) || !(opts->eps_tol > 0.0))
        return set_error(FPS_ERR_INVALID_ARG, "eps_tol must be finite and > 0");
    if (!std::isfinite(opts->e_r) || opts->e_r < 0.0) return set_error(FPS_ERR_INVALID_ARG, "e_r must be finite and >= 0");
    const int K = opts->K > 0 ? opts->K : 10;
    if ((K % 2) != 0 || K < 2) return set_error(FPS_ERR_INVALID_ARG, "K must be even and >= 2");
    if (opts->max_alg1_iters < 0) return set_error(FPS_ERR_INVALID_ARG, "max_alg1_iters must be >= 0");
    for (int i = 0; i < L; ++i)
        if (!std::isfinite(a[i])) return set_error(FPS_ERR_INVALID_ARG, "coefficient %d is not finite", i);
    FPS_TRY(check_view(Z, "Z", -1));
    if (Z->n >= kColSumMaxN)
        return set_error(FPS_ERR_CAPACITY, "n = %lld: series mode (Algorithm 1) needs n < 2^24", (long long)Z->n);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!(flags & FPS_FLAG_NO_VALIDATE)) FPS_TRY(validate_on_device(Z, "Z", st));
    // Algorithm 2 steps 1-3
    std::vector<double> z((size_t)L);
    {
        EstWork w;
        FPS_TRY(w.init(Z, st));
        FPS_TRY(power_norm_bounds(w, Z, K, L - 1, z.data(), st));
    }
    int N = 0, q = 0;
    double tail = 0.0;
    FPS_TRY(series_degree(a, L, z.data(), opts->eps_tol, &N, &q, &tail));
    if (q > FPS_MAX_S) return set_error(FPS_ERR_CAPACITY, "q = %d exceeds FPS_MAX_S", q);
    const double budget = opts->eps_tol - tail;
    fps_filter_opts fo{};
    fo.filter = FPS_FILTER_ADAPTIVE;
    fo.max_alg1_iters = opts->max_alg1_iters;
    fo.alg1_device_iters = opts->alg1_device_iters;
    fo.eps = budget;
    fo.e_r = opts->e_r;
    fo.znorm = z.data();
    fps_plan pl = nullptr;
    FPS_TRY(fps_plan_create_ex(&pl, Z, a, N - 1, q, &fo, flags | FPS_FLAG_NO_VALIDATE, stream));
    pl->series = true;
    pl->series_N = N;
    pl->series_q = q;
    pl->series_tail = tail;
    pl->series_budget = budget;
    pl->series_z = std::move(z);
    *out = pl;
    return FPS_OK;
}

fps_status fps_plan_series_info(fps_plan p, int32_t* N, int32_t* q, double* tail, double* budget, double* z)
{
    if (!p) return set_error(FPS_ERR_INVALID_ARG, "plan is NULL");
    if (!p->series) return set_error(FPS_ERR_INVALID_ARG, "not a series plan");
    if (N) *N = p->series_N;
    if (q) *q = p->series_q;
    if (tail) *tail = p->series_tail;
    if (budget) *budget = p->series_budget;
    if (z) std::memcpy(z, p->series_z.data(), sizeof(double) * p->series_z.size());
    return FPS_OK;
}

}  // extern "C"

// ===========================================================================
// Batch, and its autotuner of the block size
// ===========================================================================

namespace {

// Instances joined into one block-diagonal CSR: instance j's rows follow
// those of instances 0..j-1, its columns shifted alike, with its threshold
// on each of its rows.
struct Joined {
    std::vector<int> members;   // item indices
    std::vector<int64_t> base;  // first row of each member, and the total
    int64_t rows = 0, nnz = 0;
    DevBuf rp, col, val, tau_row, dbase;

    fps_status build(const fps_batch_item* items, hipStream_t st)
    {
        const int cnt = (int)members.size();
        base.assign(1, 0);
        rows = nnz = 0;
        std::vector<BatchSrc> src((size_t)cnt);
        for (int j = 0; j < cnt; ++j) {
            const fps_batch_item& it = items[members[(size_t)j]];
            src[(size_t)j] = BatchSrc{it.Z.row_ptr, it.Z.col, it.Z.val, nnz, it.tau};
            nnz += it.Z.nnz;
            rows += it.Z.n;
            base.push_back(rows);
        }
        if (rows > FPS_MAX_N) return set_error(FPS_ERR_CAPACITY, "a batch group has %lld rows", (long long)rows);
        DevBuf dsrc;
        FPS_TRY(dsrc.ensure(sizeof(BatchSrc) * (size_t)cnt));
        FPS_TRY(dbase.ensure(sizeof(int64_t) * (size_t)(cnt + 1)));
        FPS_TRY(rp.ensure(sizeof(int64_t) * (size_t)(rows + 1)));
        FPS_TRY(col.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1)));
        FPS_TRY(val.ensure(sizeof(double) * (size_t)std::max<int64_t>(nnz, 1)));
        FPS_TRY(tau_row.ensure(sizeof(double) * (size_t)rows));
        HIP_TRY(hipMemcpyAsync(dsrc.p, src.data(), sizeof(BatchSrc) * (size_t)cnt, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(dbase.p, base.data(), sizeof(int64_t) * (size_t)(cnt + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(launch_batch_join(dsrc.as<BatchSrc>(), dbase.as<int64_t>(), cnt, rows, rp.as<int64_t>(),
                                  col.as<int32_t>(), val.as<double>(), tau_row.as<double>(), st));
        HIP_TRY(hipStreamSynchronize(st));  // dsrc is released on return
        return FPS_OK;
    }

    fps_csr_view view() const { return fps_csr_view{rows, nnz, rp.as<int64_t>(), col.as<int32_t>(), val.as<double>()}; }
};

// Multiply-adds of one sizing evaluation with block size s, per member of a
// joined set (exact integers: each row's count is added by one thread, the
// per-member sums are integer atomics).
fps_status measure_products(Joined& J, const std::vector<double>& c, int m, int s, uint64_t flags, hipStream_t st,
                            std::vector<int64_t>& out)
{
    const int cnt = (int)J.members.size();
    fps_plan p = nullptr;
    const fps_csr_view v = J.view();
    FPS_TRY(fps_plan_create(&p, &v, c.data(), m, s, 0.0, flags | FPS_FLAG_NO_VALIDATE,
                            reinterpret_cast<fps_stream>(st)));
    std::unique_ptr<fps_plan_s, void (*)(fps_plan)> guard(p, fps_plan_destroy);
    DevBuf acc, sums;
    FPS_TRY(acc.ensure(sizeof(int64_t) * (size_t)J.rows));
    FPS_TRY(sums.ensure(sizeof(unsigned long long) * (size_t)cnt));
    HIP_TRY(launch_fill_u64(reinterpret_cast<unsigned long long*>(acc.p), J.rows, 0ull, st));
    HIP_TRY(launch_fill_u64(sums.as<unsigned long long>(), cnt, 0ull, st));
    p->tau_row = J.tau_row.as<double>();
    p->prod_acc = acc.as<int64_t>();
    FPS_TRY(fps_eval(p, reinterpret_cast<fps_stream>(st)));
    FPS_TRY(finish(p));
    HIP_TRY(launch_batch_instance_sum(acc.as<int64_t>(), J.dbase.as<int64_t>(), cnt, J.rows,
                                      sums.as<unsigned long long>(), st));
    std::vector<unsigned long long> h((size_t)cnt);
    HIP_TRY(hipMemcpyAsync(h.data(), sums.p, sizeof(unsigned long long) * (size_t)cnt, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    out.assign(h.begin(), h.end());
    return FPS_OK;
}

}  // namespace

struct fps_batch_s {
    struct Item {
        int group = -1, member = -1;
        int64_t n = 0, nnz = 0;
        int m = 0, s = 0;
        double tau = 0.0;
        bool tuned = false;
        std::vector<int64_t> products;  // tuned: multiply-adds measured for s = s_lo .. s_hi
    };
    struct Group {
        int m = 0, s = 0;
        std::vector<double> c;
        Joined J;
        DevBuf dbounds;
        fps_plan plan = nullptr;
        std::vector<int64_t> bounds;  // [2 j, 2 j + 1): member j's entries in the joined result
        hipStream_t fork = nullptr;
        hipEvent_t joined = nullptr;
    };
    std::vector<Item> items;
    std::deque<Group> groups;  // stable addresses (DevBuf is not movable)
    uint64_t flags = 0;
    int s_lo = 0, s_hi = 0;
    bool sized = false;
    bool use_graph = true;
    hipStream_t cap = nullptr;
    hipEvent_t forked = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last_stream = nullptr;
    int64_t evals = 0, graph_launches = 0, collected = -1;

    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }

    ~fps_batch_s()
    {
        if (evals) (void)hipStreamSynchronize(last_stream);
        drop_graph();
        for (Group& g : groups) {
            if (g.plan) fps_plan_destroy(g.plan);
            if (g.fork) (void)hipStreamDestroy(g.fork);
            if (g.joined) (void)hipEventDestroy(g.joined);
        }
        if (cap) (void)hipStreamDestroy(cap);
        if (forked) (void)hipEventDestroy(forked);
    }

    int64_t plan_resizes() const
    {
        int64_t t = 0;
        for (const Group& g : groups) t += g.plan->resizes;
        return t;
    }

    // Every group's evaluation (no sizing) on its own branch off `s`: fork on
    // an event, join on the groups' events.  Every branch is joined even if a
    // group fails, so that a capture on `s` always ends with no stream left
    // capturing; the first failure is returned.
    fps_status enqueue_groups(hipStream_t s)
    {
        HIP_TRY(hipEventRecord(forked, s));
        fps_status first = FPS_OK;
        for (Group& g : groups) {
            HIP_TRY(hipStreamWaitEvent(g.fork, forked, 0));
            if (first == FPS_OK) first = g.plan->run_eval(g.fork, false);
            HIP_TRY(hipEventRecord(g.joined, g.fork));
            HIP_TRY(hipStreamWaitEvent(s, g.joined, 0));
        }
        return first;
    }

    // Captures enqueue_groups into a graph; if capture or instantiation
    // fails, the batch keeps using ordinary launches.
    void capture()
    {
        drop_graph();
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            use_graph = false;
            return;
        }
        const fps_status st = enqueue_groups(cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cap, &g);
        if (st != FPS_OK || e != hipSuccess || !g) {
            (void)hipGetLastError();
            if (g) (void)hipGraphDestroy(g);
            use_graph = false;
            return;
        }
        graph = g;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGetLastError();
            drop_graph();
            use_graph = false;
        }
    }

    // After an evaluation: every group finished (a flagged group is run
    // again with sizing, which invalidates the graph) and the members'
    // bounds in the joined results read.
    fps_status collect()
    {
        if (collected == evals) return FPS_OK;
        const int64_t before = plan_resizes();
        for (Group& g : groups) FPS_TRY(finish(g.plan));
        if (plan_resizes() != before) drop_graph();
        for (Group& g : groups) {
            const int cnt = (int)g.J.members.size();
            HIP_TRY(launch_batch_bounds(g.plan->result.rp.as<int64_t>(), g.J.dbase.as<int64_t>(), cnt,
                                        g.dbounds.as<int64_t>(), g.plan->last_stream));
            g.bounds.resize(2 * (size_t)cnt);
            HIP_TRY(hipMemcpyAsync(g.bounds.data(), g.dbounds.p, sizeof(int64_t) * g.bounds.size(),
                                   hipMemcpyDeviceToHost, g.plan->last_stream));
            HIP_TRY(hipStreamSynchronize(g.plan->last_stream));
        }
        collected = evals;
        return FPS_OK;
    }
};

extern "C" {

fps_status fps_batch_create(fps_batch* out, const fps_batch_item* items, int32_t count, int32_t s_lo, int32_t s_hi,
                            uint64_t flags, fps_stream stream)
{
    g_last_error.clear();
    if (!out) return set_error(FPS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!items || count < 1) return set_error(FPS_ERR_INVALID_ARG, "need at least one item");
    if (flags & FPS_FLAG_DROP_STATS) return set_error(FPS_ERR_INVALID_ARG, "FPS_FLAG_DROP_STATS is not supported by batches");
    if (s_lo < 0 || s_hi < s_lo || s_hi > FPS_MAX_S || (s_lo == 0 && s_hi != 0))
        return set_error(FPS_ERR_INVALID_ARG, "autotuner range [%d, %d] invalid", s_lo, s_hi);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    for (int i = 0; i < count; ++i) {
        const fps_batch_item& it = items[i];
        FPS_TRY(check_view(&it.Z, "batch item Z", -1));
        if (!it.coeffs) return set_error(FPS_ERR_INVALID_ARG, "item %d: coeffs is NULL", i);
        if (it.m < 0) return set_error(FPS_ERR_INVALID_ARG, "item %d: m must be >= 0", i);
        if (it.s < 0 || it.s > FPS_MAX_S) return set_error(FPS_ERR_INVALID_ARG, "item %d: s out of range", i);
        if (!std::isfinite(it.tau) || it.tau < 0.0) return set_error(FPS_ERR_INVALID_ARG, "item %d: bad tau", i);
        for (int k = 0; k <= it.m; ++k)
            if (!std::isfinite(it.coeffs[k])) return set_error(FPS_ERR_INVALID_ARG, "item %d: coefficient %d", i, k);
    }
    if (!(flags & FPS_FLAG_NO_VALIDATE)) {
        DevBuf flag;
        FPS_TRY(flag.ensure(sizeof(unsigned long long) * (size_t)count));
        unsigned long long* fl = flag.as<unsigned long long>();
        HIP_TRY(launch_fill_u64(fl, count, 0ull, st));
        for (int i = 0; i < count; ++i)
            HIP_TRY(launch_validate_csr(items[i].Z.row_ptr, items[i].Z.col, items[i].Z.val, items[i].Z.n,
                                        items[i].Z.nnz, fl + i, st));
        std::vector<unsigned long long> h((size_t)count);
        HIP_TRY(hipMemcpyAsync(h.data(), fl, sizeof(unsigned long long) * (size_t)count, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int i = 0; i < count; ++i)
            if (h[(size_t)i]) return set_error(FPS_ERR_BAD_CSR, "batch item %d is not a canonical CSR", i);
    }
    std::unique_ptr<fps_batch_s> b(new (std::nothrow) fps_batch_s());
    if (!b) return set_error(FPS_ERR_OUT_OF_MEMORY, "host allocation failed");
    b->flags = flags & (FPS_FLAG_NO_SKIP | FPS_FLAG_FORCE_GLOBAL);
    b->use_graph = !(flags & FPS_BATCH_NO_GRAPH);
    b->s_lo = s_lo;
    b->s_hi = s_hi;
    b->items.resize((size_t)count);
    for (int i = 0; i < count; ++i) {
        auto& x = b->items[(size_t)i];
        x.n = items[i].Z.n;
        x.nnz = items[i].Z.nnz;
        x.m = items[i].m;
        x.tau = items[i].tau;
        x.s = items[i].s;
    }
    auto same_series = [&](int i, int j) {
        return items[i].m == items[j].m &&
               std::memcmp(items[i].coeffs, items[j].coeffs, sizeof(double) * (size_t)(items[i].m + 1)) == 0;
    };
    // Autotuner: items without s, by families of the same series, take the
    // block size with the fewest multiply-adds in one sizing evaluation of
    // the family per candidate (ties: the smaller s).
    {
        std::vector<int> family((size_t)count, -1);
        std::vector<int> heads;
        for (int i = 0; i < count; ++i) {
            if (items[i].s != 0) continue;
            for (int h : heads)
                if (same_series(h, i)) {
                    family[(size_t)i] = h;
                    break;
                }
            if (family[(size_t)i] < 0) {
                family[(size_t)i] = i;
                heads.push_back(i);
            }
        }
        for (int h : heads) {
            Joined J;
            for (int i = 0; i < count; ++i)
                if (family[(size_t)i] == h) J.members.push_back(i);
            FPS_TRY(J.build(items, st));
            int lo = s_lo, hi = s_hi;
            if (lo == 0) {
                int r = 0;
                while ((r + 1) * (r + 1) <= items[h].m) ++r;
                lo = std::max(1, r - 1);
                hi = std::min(FPS_MAX_S, std::max(lo, r + 1));
            }
            const std::vector<double> c(items[h].coeffs, items[h].coeffs + items[h].m + 1);
            for (int s = lo; s <= hi; ++s) {
                std::vector<int64_t> prod;
                FPS_TRY(measure_products(J, c, items[h].m, s, b->flags, st, prod));
                for (size_t j = 0; j < J.members.size(); ++j) {
                    auto& x = b->items[(size_t)J.members[j]];
                    x.products.push_back(prod[j]);
                    if (s == lo || prod[j] < x.products[(size_t)(x.s - lo)]) x.s = s;
                    x.tuned = true;
                }
            }
        }
    }
    // groups: same m, s and coefficients
    std::vector<int> head_of;  // first item of each group
    for (int i = 0; i < count; ++i) {
        auto& x = b->items[(size_t)i];
        int gi = -1;
        for (size_t k = 0; k < head_of.size(); ++k)
            if (b->items[(size_t)head_of[k]].s == x.s && same_series(head_of[k], i)) {
                gi = (int)k;
                break;
            }
        if (gi < 0) {
            b->groups.emplace_back();
            auto& g = b->groups.back();
            g.m = x.m;
            g.s = x.s;
            g.c.assign(items[i].coeffs, items[i].coeffs + x.m + 1);
            head_of.push_back(i);
            gi = (int)b->groups.size() - 1;
        }
        auto& g = b->groups[(size_t)gi];
        x.group = gi;
        x.member = (int)g.J.members.size();
        g.J.members.push_back(i);
    }
    HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&b->forked, hipEventDisableTiming));
    for (auto& g : b->groups) {
        FPS_TRY(g.J.build(items, st));
        FPS_TRY(g.dbounds.ensure(sizeof(int64_t) * 2 * g.J.members.size()));
        const fps_csr_view v = g.J.view();
        FPS_TRY(fps_plan_create(&g.plan, &v, g.c.data(), g.m, g.s, 0.0, b->flags | FPS_FLAG_NO_VALIDATE, stream));
        g.plan->tau_row = g.J.tau_row.as<double>();
        HIP_TRY(hipStreamCreateWithFlags(&g.fork, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&g.joined, hipEventDisableTiming));
    }
    *out = b.release();
    return FPS_OK;
}

fps_status fps_batch_eval(fps_batch b, fps_stream stream)
{
    if (!b) return set_error(FPS_ERR_INVALID_ARG, "batch is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!b->sized) {
        // sizing evaluation, group after group (host reads per stage)
        for (auto& g : b->groups) FPS_TRY(fps_eval(g.plan, stream));
        b->sized = true;
    } else {
        // the first evaluation after sizing runs with ordinary launches (it may
        // still grow a buffer, e.g. the fixed stride of a stage whose rows were
        // all empty, which a capture cannot do); later ones replay the graph
        if (b->use_graph && !b->exec && b->evals >= 2) b->capture();
        if (b->use_graph && b->exec) {
            HIP_TRY(hipGraphLaunch(b->exec, s));
            b->graph_launches++;
        } else {
            FPS_TRY(b->enqueue_groups(s));
        }
        for (auto& g : b->groups) {
            g.plan->last_stream = s;
            g.plan->evals++;
            g.plan->evaluated = true;
        }
    }
    b->last_stream = s;
    b->evals++;
    return FPS_OK;
}

fps_status fps_batch_result_nnz(fps_batch b, int32_t i, int64_t* nnz)
{
    if (!b || !nnz) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    if (i < 0 || i >= (int32_t)b->items.size()) return set_error(FPS_ERR_INVALID_ARG, "item index out of range");
    if (!b->evals) return set_error(FPS_ERR_NOT_READY, "no evaluation has run on this batch");
    FPS_TRY(b->collect());
    const auto& x = b->items[(size_t)i];
    const auto& g = b->groups[(size_t)x.group];
    *nnz = g.bounds[2 * (size_t)x.member + 1] - g.bounds[2 * (size_t)x.member];
    return FPS_OK;
}

fps_status fps_batch_result_copy(fps_batch b, int32_t i, int64_t* row_ptr, int32_t* col, double* val,
                                 fps_stream stream)
{
    if (!b || !row_ptr) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    int64_t nnz = 0;
    FPS_TRY(fps_batch_result_nnz(b, i, &nnz));
    if (nnz > 0 && (!col || !val)) return set_error(FPS_ERR_INVALID_ARG, "null col/val with nnz > 0");
    const auto& x = b->items[(size_t)i];
    const auto& g = b->groups[(size_t)x.group];
    const int64_t row0 = g.J.base[(size_t)x.member];
    const int64_t p0 = g.bounds[2 * (size_t)x.member];
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(launch_batch_extract(g.plan->result.rp.as<int64_t>(), g.plan->result.col.as<int32_t>(), row0, x.n, p0,
                                 nnz, (int32_t)row0, row_ptr, col, s));
    if (nnz > 0)
        HIP_TRY(hipMemcpyAsync(val, g.plan->result.val.as<double>() + p0, sizeof(double) * (size_t)nnz,
                               hipMemcpyDeviceToDevice, s));
    return FPS_OK;
}

fps_status fps_batch_get_stats(fps_batch b, fps_batch_stats* st)
{
    if (!b || !st) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    std::memset(st, 0, sizeof(*st));
    st->count = (int32_t)b->items.size();
    st->groups = (int32_t)b->groups.size();
    st->graph = (b->use_graph && b->exec) ? 1 : 0;
    st->evals = b->evals;
    st->graph_launches = b->graph_launches;
    for (const auto& g : b->groups) st->rows += g.J.rows;
    if (!b->evals) return FPS_OK;
    FPS_TRY(b->collect());
    st->resizes = b->plan_resizes();
    for (auto& g : b->groups) {
        fps_stats ps;
        FPS_TRY(fps_get_stats(g.plan, &ps));
        st->nnz_out += ps.nnz_out;
        st->products += ps.products;
        st->bytes_algorithmic += ps.bytes_algorithmic;
    }
    return FPS_OK;
}

fps_status fps_batch_item_info(fps_batch b, int32_t i, int32_t* s, int32_t* group, int64_t* products)
{
    if (!b) return set_error(FPS_ERR_INVALID_ARG, "batch is NULL");
    if (i < 0 || i >= (int32_t)b->items.size()) return set_error(FPS_ERR_INVALID_ARG, "item index out of range");
    const auto& x = b->items[(size_t)i];
    if (s) *s = x.s;
    if (group) *group = x.group;
    if (products)
        for (size_t k = 0; k < x.products.size(); ++k) products[k] = x.products[k];
    return FPS_OK;
}

void fps_batch_destroy(fps_batch b) { delete b; }

}  // extern "C"

// ===========================================================================
// Server
// ===========================================================================

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First reservation of a request: the plan's per-row arrays and, per stage,
// a slack matrix for rows of about (s + 1) times Z's entries per row, at
// 24 bytes an entry (value, column, structure word).  A request that needs
// more is run again with a larger reservation.
size_t first_reservation(int64_t n, int64_t nnz, int m, int s)
{
    Schedule sc;
    make_schedule(m, s, &sc);
    const double stages = (double)(sc.J + sc.b + 2);
    const double per_row = (double)nnz / (double)std::max<int64_t>(n, 1);
    const double entries = (double)n * std::max(1.0, per_row) * (double)(s + 1);
    const double bytes = (double)n * 160.0 + stages * (entries * 24.0 + (double)n * 40.0);
    return (size_t)std::min(bytes, 1e18);
}

}  // namespace

struct fps_server_s {
    struct Req {
        int64_t id = 0;
        fps_csr_view Z{};
        std::vector<double> c;
        int m = 0, s = 0;
        double tau = 0.0;
        int state = FPS_REQ_QUEUED;
        fps_status status = FPS_OK;
        std::string error;
        int attempts = 0;
        fps_server_s* sv = nullptr;  // the server (for growing the reservation in place)
        size_t reserve = 0, held = 0, peak = 0;
        int64_t nnz_out = 0;
        DevBuf rp, col, val;  // the result, kept until release
        hipEvent_t copied = nullptr;  // recorded after the last copy out of the result
        int64_t t_submit = 0, t_start = 0, t_done = 0;
        ~Req()
        {
            if (copied) {
                (void)hipEventSynchronize(copied);
                (void)hipEventDestroy(copied);
            }
        }
    };

    DevPool pool;  // first member: it outlives every buffer handed out from it
    fps_server_opts o{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> queue;
    std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
    int64_t next_id = 1;
    size_t reserved = 0, peak_reserved = 0;
    int running = 0, peak_running = 0;
    int64_t submitted = 0, completed = 0, failed = 0, retries = 0, refused = 0, grows = 0;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;

    // Raises the reservation of running request r to at least `need` bytes
    // (a quarter more where the budget allows, so that a plan grows in few
    // steps) if the budget has room beside everything else reserved or held;
    // the plan's account `a` (if any) follows.  Called by the request's own
    // worker (no lock held).
    bool grow(Req* r, size_t need, MemAcct* a)
    {
        size_t keep = 0;
        {
            std::lock_guard<std::mutex> lk(mu);
            const size_t budget = (size_t)o.hbm_budget;
            const size_t others = reserved - r->reserve;
            if (need > budget || others > budget - need) return false;
            const size_t want = std::min(budget - others, need + need / 4);
            reserved = others + want;
            peak_reserved = std::max(peak_reserved, reserved);
            r->reserve = want;
            if (a) a->cap = want;
            grows++;
            keep = budget - reserved;
        }
        // pooled free blocks count against the budget as well
        if (!o.fake_backend) pool.trim(keep);
        return true;
    }

    static bool extend_hook(void* ctx, MemAcct* a, size_t need)
    {
        Req* r = static_cast<Req*>(ctx);
        return r->sv->grow(r, need, a);
    }

    // Runs one attempt of a request on `st` (no lock held).
    void execute(Req* r, hipStream_t st)
    {
        r->status = FPS_OK;
        r->error.clear();
        if (o.fake_backend) {
            r->peak = (size_t)r->Z.n * 100;
            if (r->peak > r->reserve && (o.no_grow || !grow(r, r->peak, nullptr))) {
                r->status = FPS_ERR_CAPACITY;
                r->error = "fake backend: reservation too small";
                return;
            }
            std::this_thread::sleep_for(std::chrono::microseconds(r->Z.n));
            r->held = 0;
            r->nnz_out = 0;
            return;
        }
        fps_filter_opts fo{};
        fo.filter = FPS_FILTER_FIXED;
        fo.tau = r->tau;
        fps_plan p = nullptr;
        fps_status stt = plan_create_limited(&p, &r->Z, r->c.data(), r->m, r->s, &fo, o.flags,
                                             reinterpret_cast<fps_stream>(st), r->reserve,
                                             o.no_grow ? nullptr : &extend_hook, r);
        if (stt == FPS_OK) p->eng.one_shot = true;  // one evaluation per request
        if (stt == FPS_OK) stt = fps_eval(p, reinterpret_cast<fps_stream>(st));
        if (stt == FPS_OK) stt = finish(p);
        if (stt == FPS_OK) {
            // keep only the result, in buffers of the server's own
            const int64_t n = r->Z.n;
            int64_t nnz = 0;
            stt = fps_result_nnz(p, &nnz);
            // the copy exists beside the plan for a moment: it must fit the
            // reservation too (its three buffers as the pool hands them out,
            // rounded up to the pool's size classes)
            auto cls = [](size_t b) { return DevPool::size_class(std::max<size_t>(b, 256)); };
            const size_t e = (size_t)std::max<int64_t>(nnz, 1);
            const size_t copy = cls(sizeof(int64_t) * (size_t)(n + 1)) + cls(sizeof(int32_t) * e) + cls(sizeof(double) * e);
            if (stt == FPS_OK && !p->acct.admit(copy))
                stt = set_error(FPS_ERR_CAPACITY, "the result copy does not fit the reservation");
            if (stt == FPS_OK) stt = r->rp.ensure(sizeof(int64_t) * (size_t)(n + 1));
            if (stt == FPS_OK) stt = r->col.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
            if (stt == FPS_OK) stt = r->val.ensure(sizeof(double) * (size_t)std::max<int64_t>(nnz, 1));
            if (stt == FPS_OK)
                stt = fps_result_copy(p, r->rp.as<int64_t>(), r->col.as<int32_t>(), r->val.as<double>(),
                                      reinterpret_cast<fps_stream>(st));
            if (stt == FPS_OK && hipStreamSynchronize(st) != hipSuccess) {
                (void)hipGetLastError();
                stt = set_error(FPS_ERR_HIP, "stream synchronisation failed");
            }
            r->nnz_out = nnz;
            r->held = r->rp.bytes + r->col.bytes + r->val.bytes;
        }
        if (p) r->peak = std::max(p->acct.peak, p->acct.used + r->rp.bytes + r->col.bytes + r->val.bytes);
        if (stt != FPS_OK) {
            r->error = g_last_error;
            r->rp.release();
            r->col.release();
            r->val.release();
            r->held = 0;
        }
        r->status = stt;
        if (p) fps_plan_destroy(p);
    }

    void worker(int k)
    {
        if (!o.fake_backend) (void)hipSetDevice(device);
        t_pool = o.fake_backend ? nullptr : &pool;
        for (;;) {
            Req* r = nullptr;
            size_t keep = SIZE_MAX;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    return stopping || (!queue.empty() && reserved + queue.front()->reserve <= (size_t)o.hbm_budget);
                });
                if (stopping) return;
                r = queue.front();
                queue.pop_front();
                reserved += r->reserve;
                peak_reserved = std::max(peak_reserved, reserved);
                running++;
                peak_running = std::max(peak_running, running);
                r->state = FPS_REQ_RUNNING;
                r->attempts++;
                r->t_start = now_ns();
                // pooled free blocks count against the budget as well
                keep = (size_t)o.hbm_budget - reserved;
            }
            if (!o.fake_backend) pool.trim(keep);
            execute(r, o.fake_backend ? nullptr : streams[(size_t)k]);
            {
                std::lock_guard<std::mutex> lk(mu);
                running--;
                reserved -= r->reserve;
                if (r->status == FPS_ERR_CAPACITY && r->reserve < (size_t)o.hbm_budget && r->attempts < 16) {
                    // the reservation was too small: back to the head with more
                    r->reserve = (size_t)std::min<double>((double)o.hbm_budget, 4.0 * (double)r->reserve);
                    r->state = FPS_REQ_QUEUED;
                    queue.push_front(r);
                    retries++;
                } else {
                    r->t_done = now_ns();
                    if (r->status == FPS_OK) {
                        r->state = FPS_REQ_DONE;
                        reserved += r->held;
                        peak_reserved = std::max(peak_reserved, reserved);
                        completed++;
                    } else {
                        r->state = FPS_REQ_FAILED;
                        failed++;
                    }
                }
            }
            cv_work.notify_all();
            cv_done.notify_all();
        }
    }

    Req* find(int64_t id)
    {
        auto it = reqs.find(id);
        return it == reqs.end() ? nullptr : it->second.get();
    }

    ~fps_server_s()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            stopping = true;
            for (Req* r : queue) {
                r->state = FPS_REQ_FAILED;
                r->status = FPS_ERR_NOT_READY;
                r->t_done = now_ns();
            }
            queue.clear();
        }
        cv_work.notify_all();
        cv_done.notify_all();
        for (auto& t : workers)
            if (t.joinable()) t.join();
        if (!o.fake_backend) (void)hipDeviceSynchronize();
        reqs.clear();
        for (hipStream_t s : streams) (void)hipStreamDestroy(s);
    }
};

extern "C" {

fps_status fps_server_create(fps_server* out, const fps_server_opts* opts)
{
    g_last_error.clear();
    if (!out || !opts) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (opts->slots < 1 || opts->slots > 64) return set_error(FPS_ERR_INVALID_ARG, "slots must be in [1, 64]");
    if (opts->hbm_budget <= 0) return set_error(FPS_ERR_INVALID_ARG, "hbm_budget must be > 0");
    if (opts->max_queue < 0) return set_error(FPS_ERR_INVALID_ARG, "max_queue must be >= 0");
    if (opts->flags & ~(uint64_t)(FPS_FLAG_NO_VALIDATE | FPS_FLAG_NO_SKIP | FPS_FLAG_DENSE | FPS_FLAG_DENSE_EXACT))
        return set_error(FPS_ERR_INVALID_ARG, "unsupported server flags");
    std::unique_ptr<fps_server_s> sv(new (std::nothrow) fps_server_s());
    if (!sv) return set_error(FPS_ERR_OUT_OF_MEMORY, "host allocation failed");
    sv->o = *opts;
    if (sv->o.max_queue == 0) sv->o.max_queue = 4096;
    if (!opts->fake_backend) {
        HIP_TRY(hipGetDevice(&sv->device));
        for (int k = 0; k < opts->slots; ++k) {
            hipStream_t s = nullptr;
            HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            sv->streams.push_back(s);
        }
    }
    fps_server_s* raw = sv.get();
    for (int k = 0; k < opts->slots; ++k) sv->workers.emplace_back([raw, k] { raw->worker(k); });
    *out = sv.release();
    return FPS_OK;
}

fps_status fps_server_submit(fps_server sv, const fps_csr_view* Z, const double* coeffs, int32_t m, int32_t s,
                             double tau, int64_t reserve_hint, int64_t* ticket)
{
    g_last_error.clear();
    if (!sv || !ticket || !coeffs) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    FPS_TRY(check_view(Z, "Z", -1));
    if (m < 0) return set_error(FPS_ERR_INVALID_ARG, "m must be >= 0");
    if (s < 0 || s > FPS_MAX_S) return set_error(FPS_ERR_INVALID_ARG, "s out of range");
    if (!std::isfinite(tau) || tau < 0.0) return set_error(FPS_ERR_INVALID_ARG, "tau must be finite and >= 0");
    for (int k = 0; k <= m; ++k)
        if (!std::isfinite(coeffs[k])) return set_error(FPS_ERR_INVALID_ARG, "coefficient %d is not finite", k);
    std::unique_ptr<fps_server_s::Req> r(new (std::nothrow) fps_server_s::Req());
    if (!r) return set_error(FPS_ERR_OUT_OF_MEMORY, "host allocation failed");
    r->Z = *Z;
    r->c.assign(coeffs, coeffs + m + 1);
    r->m = m;
    r->sv = sv;
    if (s == 0) {
        s = 0;
        while ((s + 1) * (s + 1) <= m) ++s;
        s = std::min(std::max(s, 1), FPS_MAX_S);
    }
    r->s = s;
    r->tau = tau;
    r->reserve = reserve_hint > 0 ? (size_t)reserve_hint : first_reservation(Z->n, Z->nnz, m, s);
    r->reserve = std::min(r->reserve, (size_t)sv->o.hbm_budget);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stopping) return set_error(FPS_ERR_INVALID_ARG, "server is stopping");
        if ((int64_t)sv->queue.size() >= sv->o.max_queue) {
            sv->refused++;
            return set_error(FPS_ERR_CAPACITY, "server queue full (%d waiting)", sv->o.max_queue);
        }
        r->id = sv->next_id++;
        r->t_submit = now_ns();
        *ticket = r->id;
        sv->queue.push_back(r.get());
        sv->reqs.emplace(r->id, std::move(r));
        sv->submitted++;
    }
    sv->cv_work.notify_all();
    return FPS_OK;
}

fps_status fps_server_wait(fps_server sv, int64_t ticket, int64_t timeout_ms, int32_t* state)
{
    if (!sv) return set_error(FPS_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    fps_server_s::Req* r = sv->find(ticket);
    if (!r) return set_error(FPS_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    auto finished = [&] { return r->state == FPS_REQ_DONE || r->state == FPS_REQ_FAILED; };
    if (timeout_ms < 0)
        sv->cv_done.wait(lk, finished);
    else
        sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished);
    if (state) *state = r->state;
    return FPS_OK;
}

fps_status fps_server_result_nnz(fps_server sv, int64_t ticket, int64_t* nnz)
{
    if (!sv || !nnz) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    fps_server_s::Req* r = sv->find(ticket);
    if (!r) return set_error(FPS_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    if (r->state != FPS_REQ_DONE) return set_error(FPS_ERR_NOT_READY, "request %lld is not done", (long long)ticket);
    *nnz = r->nnz_out;
    return FPS_OK;
}

fps_status fps_server_result_copy(fps_server sv, int64_t ticket, int64_t* row_ptr, int32_t* col, double* val,
                                  fps_stream stream)
{
    if (!sv || !row_ptr) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    fps_server_s::Req* r = sv->find(ticket);
    if (!r) return set_error(FPS_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    if (r->state != FPS_REQ_DONE) return set_error(FPS_ERR_NOT_READY, "request %lld is not done", (long long)ticket);
    if (sv->o.fake_backend) return set_error(FPS_ERR_INVALID_ARG, "the fake backend has no results");
    if (r->nnz_out > 0 && (!col || !val)) return set_error(FPS_ERR_INVALID_ARG, "null col/val with nnz > 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(row_ptr, r->rp.p, sizeof(int64_t) * (size_t)(r->Z.n + 1), hipMemcpyDeviceToDevice, s));
    if (r->nnz_out > 0) {
        HIP_TRY(hipMemcpyAsync(col, r->col.p, sizeof(int32_t) * (size_t)r->nnz_out, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(val, r->val.p, sizeof(double) * (size_t)r->nnz_out, hipMemcpyDeviceToDevice, s));
    }
    if (!r->copied) HIP_TRY(hipEventCreateWithFlags(&r->copied, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(r->copied, s));
    return FPS_OK;
}

fps_status fps_server_release(fps_server sv, int64_t ticket)
{
    if (!sv) return set_error(FPS_ERR_INVALID_ARG, "server is NULL");
    std::unique_ptr<fps_server_s::Req> gone;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        if (it == sv->reqs.end()) return set_error(FPS_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
        fps_server_s::Req* r = it->second.get();
        if (r->state != FPS_REQ_DONE && r->state != FPS_REQ_FAILED)
            return set_error(FPS_ERR_NOT_READY, "request %lld is still queued or running", (long long)ticket);
        sv->reserved -= r->held;
        gone = std::move(it->second);
        sv->reqs.erase(it);
    }
    gone.reset();  // waits for the copies out of the result, then frees it
    sv->cv_work.notify_all();
    return FPS_OK;
}

fps_status fps_server_request_info(fps_server sv, int64_t ticket, fps_server_request* out)
{
    if (!sv || !out) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    fps_server_s::Req* r = sv->find(ticket);
    if (!r) return set_error(FPS_ERR_INVALID_ARG, "unknown ticket %lld", (long long)ticket);
    out->state = r->state;
    out->status = r->status;
    out->attempts = r->attempts;
    out->s = r->s;
    out->n = r->Z.n;
    out->reserve = (int64_t)r->reserve;
    out->held = (int64_t)r->held;
    out->peak = (int64_t)r->peak;
    out->t_submit_ns = r->t_submit;
    out->t_start_ns = r->t_start;
    out->t_done_ns = r->t_done;
    return FPS_OK;
}

fps_status fps_server_get_stats(fps_server sv, fps_server_stats* out)
{
    if (!sv || !out) return set_error(FPS_ERR_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->failed = sv->failed;
    out->retries = sv->retries;
    out->refused = sv->refused;
    out->running = sv->running;
    out->queued = (int32_t)sv->queue.size();
    out->slots = sv->o.slots;
    out->peak_running = sv->peak_running;
    out->reserved = (int64_t)sv->reserved;
    out->peak_reserved = (int64_t)sv->peak_reserved;
    out->budget = sv->o.hbm_budget;
    out->grows = sv->grows;
    return FPS_OK;
}

void fps_server_destroy(fps_server sv) { delete sv; }

}  // extern "C"
