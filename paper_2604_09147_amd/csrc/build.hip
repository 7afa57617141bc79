// Construction of an H_h handle on the GPU: Alg. 1 (compression of every
// admissible block with target accuracy eps), Alg. 5 (norms from singular
// values) and Alg. 3 (per-block storage precision), followed by the layout of
// the product kernels' tasks.
//
// Compression: blocks with min(m, n) <= 512 take the truncated SVD of Sec. 2.2
// (Householder QR of the block, then a one-sided Jacobi SVD of the triangular
// factor); larger blocks use a randomized
// range finder (Rademacher sketch keyed by (seed, block, round), one power
// iteration, width 64 doubling while rank + 16 > width) whose truncation error
// ||H - Q Q^T H||_F^2 is summed directly, so that every block satisfies
// ||H_b - U_b V_b^T||_F <= eps ||H_b||_F (Def. of H_h(p, eps)). Batches of
// similar blocks run through rocBLAS / rocSOLVER strided-batched calls after
// zero padding to the batch maximum (zero rows and columns change neither the
// singular values nor the factors' real rows).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>

#include "handle.h"

namespace hh {

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            fail(HH_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));                 \
    } while (0)
#define RBCHK(x)                                                                           \
    do {                                                                                   \
        rocblas_status s_ = (x);                                                           \
        if (s_ != rocblas_status_success)                                                  \
            fail(s_ == rocblas_status_memory_error ? HH_ENOMEM : HH_EHIP,                  \
                 std::string(#x) + ": rocblas status " + std::to_string((int)s_));         \
    } while (0)

constexpr int EXACT_SVD_MAX = 512;
constexpr int64_t TSQR_CHUNK = 4096;      // rows of one QR kernel; taller items go through TSQR
constexpr int JACOBI_TILED_MIN_BATCH = 32;
constexpr int SKETCH_START = 64;
constexpr int OVERSAMPLE = 16;
constexpr int64_t SUM_CHUNK = 65536;
constexpr int64_t UNIT_BYTES = 1 << 20;   // default factor bytes per single-vector work unit
// The accumulation kernels address a run through one buffer descriptor with
// 32-bit byte offsets, so a run (and every slice of one) spans fewer than 2^31
// bytes: longer runs are cut by columns. HH_RUN_BYTES_MAX may lower the limit
// (to exercise the cutting at small sizes).
static int64_t run_bytes_max() {
    int64_t lim = ((int64_t)1 << 31) - 1;
    if (const char* e = getenv("HH_RUN_BYTES_MAX")) {
        const long long v = atoll(e);
        if (v > 0 && v < lim) lim = v;
    }
    return lim;
}
constexpr int64_t DOT_TASK_ELEMS = 65536;   // default elements per phase-V task
constexpr int64_t DOT_X_LDS = 4096;        // rows of x staged in LDS by dot1_kernel
// One right-hand side takes the panel tasks when a block's own phase-V tasks
// average fewer stored bytes than this (low ranks: a workgroup would finish
// after a few KB) and the panel tasks are at most half as many.
constexpr int64_t DOT_PANEL_BELOW = 32768;

void* DevMem::alloc(size_t bytes, bool zero) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(HH_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    ptrs.push_back(p);
    if (zero) {
        e = hipMemset(p, 0, bytes);
        if (e != hipSuccess) fail(HH_EHIP, std::string("hipMemset: ") + hipGetErrorString(e));
    }
    return p;
}

void DevMem::release(void* p) {
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
        (void)hipFree(p);
        ptrs.erase(it);
    }
}

void DevMem::free_all() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
}

static size_t fmt_size(int fmt) {
    return fmt == HH_FMT_FP64 ? 8 : fmt == HH_FMT_FP32 ? 4 : fmt == HH_FMT_Q43 ? 1 : 2;
}
// unit roundoffs and storage bits by HH_FMT_* (index HH_FMT_CONT unused: per block)
static const double UNIT[NFMT_CODES] = {0x1p-53, 0x1p-24, 0x1p-11, 0x1p-8, 0.0, 0x1p-4};
static const int BITS[NFMT_CODES] = {64, 32, 16, 16, 0, 8};
// Storage bits per entry of a block's format (continuum: 9 + t).
static int entry_bits(int fmt, int t) { return fmt == HH_FMT_CONT ? 9 + t : BITS[fmt]; }
// Device bytes of one stored column of P (padded) rows.
static int64_t col_bytes(int fmt, int t, int64_t P) {
    return fmt == HH_FMT_CONT ? cont_col_bytes(P, 9 + t) : P * (int64_t)fmt_size(fmt);
}

template <class T>
static T* upload(DevMem& m, const std::vector<T>& v) {
    T* d = static_cast<T*>(m.alloc(v.size() * sizeof(T) + 16, false));
    if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

// Bump allocator over one scratch buffer.
struct Carver {
    char* base;
    size_t cap;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        size_t b = (count * sizeof(T) + 255) & ~(size_t)255;
        if (off + b > cap) fail(HH_EINTERNAL, "construction scratch overflow");
        T* p = reinterpret_cast<T*>(base + off);
        off += b;
        return p;
    }
};

// Construction resources kept per device between builds: a rocBLAS handle and
// a scratch buffer of up to 2 GiB (larger scratch is allocated per build and
// freed after it). Builds in one process run one at a time.
struct BuildCache {
    rocblas_handle rb = nullptr;
    void* scratch = nullptr;
    size_t bytes = 0;
};
static std::mutex g_build_mu;
static std::map<int, BuildCache> g_build_cache;
constexpr size_t CACHED_SCRATCH_MAX = (size_t)2 << 30;

struct Builder {
    hh_handle* h;
    std::unique_lock<std::mutex> lock{g_build_mu};
    rocblas_handle rb = nullptr;
    hipStream_t st = 0;
    DevMem scratch_mem;
    char* scratch = nullptr;
    size_t scratch_bytes = 0;
    double eps2;
    std::vector<double*> store_chunks;   // fp64 factors (freed after packing unless kept)
    DevMem store;

    // per-step wall time (synchronised) when HH_VERBOSE is set
    std::map<std::string, double> tsum;
    std::chrono::steady_clock::time_point tmark;
    void tick() {
        if (!verbose()) return;
        (void)hipDeviceSynchronize();
        tmark = std::chrono::steady_clock::now();
    }
    void tock(const char* what) {
        if (!verbose()) return;
        (void)hipDeviceSynchronize();
        auto now = std::chrono::steady_clock::now();
        tsum[what] += std::chrono::duration<double>(now - tmark).count();
        tmark = now;
    }
    void report_times() {
        if (!verbose()) return;
        for (auto& kv : tsum) fprintf(stderr, "hh:   %-14s %8.2f s\n", kv.first.c_str(), kv.second);
        fflush(stderr);
    }

    // progress of the compression, printed from the batch loop when HH_VERBOSE is set
    int64_t done = 0, total_cand = 0;
    std::chrono::steady_clock::time_point t_start = std::chrono::steady_clock::now(),
                                          t_last = t_start;
    void progress(int64_t finished, const char* what, bool force = false) {
        done += finished;
        if (!verbose()) return;
        auto now = std::chrono::steady_clock::now();
        if (!force && std::chrono::duration<double>(now - t_last).count() < 10.0) return;
        t_last = now;
        fprintf(stderr, "hh: %s: %lld / %lld admissible blocks compressed, %.1f s\n", what,
                (long long)done, (long long)total_cand,
                std::chrono::duration<double>(now - t_start).count());
        fflush(stderr);
    }

    explicit Builder(hh_handle* hh) : h(hh), eps2(hh->tol * hh->tol) {}
    ~Builder() = default;          // the rocBLAS handle stays in the per-device cache

    template <class T>
    T* meta(const std::vector<T>& v, Carver& cv) {
        T* d = cv.take<T>(v.size() + 1);
        if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
        return d;
    }

    // Scratch of one batch of every candidate block at once (an upper bound of
    // what the batched compression can use).
    size_t scratch_need() const {
        double need = 0.0;
        for (const auto& r : h->blocks) {
            if (r.b.kind == HH_BLK_DIAG) continue;
            const int64_t m = r.b.ie - r.b.ib, n = r.b.je - r.b.jb;
            need += std::min(m, n) <= EXACT_SVD_MAX ? (double)exact_item_bytes(m, n)
                                                    : (double)random_item_bytes(m, n, SKETCH_START);
        }
        return need > 1e18 ? (size_t)1 << 60 : (size_t)need;
    }

    void init(size_t cap = (size_t)16 << 30) {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        BuildCache& bc = g_build_cache[dev];
        if (!bc.rb) RBCHK(rocblas_create_handle(&bc.rb));
        rb = bc.rb;
        RBCHK(rocblas_set_stream(rb, st));
        size_t freeb = 0, totalb = 0;
        HIPCHK(hipMemGetInfo(&freeb, &totalb));
        size_t want = std::min<size_t>(freeb / 5, cap);
        want = std::min(want, scratch_need() + ((size_t)64 << 20));
        if (want < ((size_t)64 << 20)) want = (size_t)64 << 20;
        if (want <= bc.bytes) {
            scratch = static_cast<char*>(bc.scratch);
            scratch_bytes = bc.bytes;
        } else if (want <= CACHED_SCRATCH_MAX) {
            void* p = nullptr;
            if (hipMalloc(&p, want) != hipSuccess) {
                (void)hipGetLastError();
                fail(HH_ENOMEM, "hipMalloc of the construction scratch failed");
            }
            if (bc.scratch) (void)hipFree(bc.scratch);
            bc.scratch = p;
            bc.bytes = want;
            scratch = static_cast<char*>(p);
            scratch_bytes = want;
        } else {
            scratch_bytes = want;
            scratch = static_cast<char*>(scratch_mem.alloc(scratch_bytes, false));
        }
    }

    // Allocate the fp64 store of a batch and record each block's factor pointers.
    double* store_for(const std::vector<int64_t>& idx, const std::vector<int>& ranks) {
        int64_t total = 0;
        for (size_t b = 0; b < idx.size(); ++b) {
            const BlockRec& r = h->blocks[idx[b]];
            total += (int64_t)ranks[b] * (r.PI + r.PJ);
        }
        double* s = static_cast<double*>(store.alloc((size_t)total * 8 + 256, true));
        int64_t off = 0;
        for (size_t b = 0; b < idx.size(); ++b) {
            BlockRec& r = h->blocks[idx[b]];
            r.u_ptr = s + off;
            off += (int64_t)ranks[b] * r.PI;
            r.v_ptr = s + off;
            off += (int64_t)ranks[b] * r.PJ;
        }
        return s;
    }

    void record_rank(int64_t bi, const RankItem& it) {
        BlockRec& r = h->blocks[bi];
        r.rank = it.rank;
        r.entry2 = it.norm2;
        r.nb2 = it.trunc2;
        r.tail = it.tail;
        r.tail_prev = it.tail_prev;
        r.fmt = HH_FMT_FP64;
    }

    // Exact SVD of blocks with min(m, n) <= EXACT_SVD_MAX: Householder QR of the
    // block (of its transpose when it is wide), then a one-sided Jacobi SVD of
    // the square triangular factor (small_svd).
    //   tall (M >= N): H = Q R, R^T J = W S  =>  H = (Q J) S W^T: U = Q J, V = W S
    //   wide (M <  N): H^T = Q R, R J = W S  =>  H = J S (Q W)^T: U = J,   V = Q W S
    // Zero padding to the batch maximum adds zero singular values only.
    void exact_batch(const std::vector<int64_t>& idx) {
        const int B = (int)idx.size();
        int64_t M = 0, N = 0;
        for (int64_t i : idx) {
            M = std::max<int64_t>(M, h->blocks[i].b.ie - h->blocks[i].b.ib);
            N = std::max<int64_t>(N, h->blocks[i].b.je - h->blocks[i].b.jb);
        }
        const bool tall = M >= N;
        const int64_t rows = tall ? M : N;
        const int s = (int)(tall ? N : M);
        const int64_t ss = (int64_t)s * s;
        const int64_t nch = (M * N + SUM_CHUNK - 1) / SUM_CHUNK;
        Carver cv{scratch, scratch_bytes};
        double* H = cv.take<double>((size_t)B * M * N);
        double* Y = tall ? H : cv.take<double>((size_t)B * M * N);
        double* Q = cv.take<double>((size_t)B * rows * s);
        double* R = cv.take<double>((size_t)B * ss);
        double* A = cv.take<double>((size_t)B * ss);
        double* J = cv.take<double>((size_t)B * ss);
        double* S = cv.take<double>((size_t)B * s);
        double* F = cv.take<double>((size_t)B * rows * s);
        double* nrm = cv.take<double>(B);
        double* part = cv.take<double>((size_t)B * nch);
        QrWork qw = qr_work(cv, B, rows, s);
        std::vector<GenItem> gi(B);
        std::vector<SumItem> si(B);
        std::vector<TransItem> ti;
        for (int b = 0; b < B; ++b) {
            const Blk& k = h->blocks[idx[b]].b;
            gi[b] = GenItem{k.ib, k.jb, k.ie - k.ib, k.je - k.jb, H + (int64_t)b * M * N, M, 0, 0};
            si[b] = SumItem{H + (int64_t)b * M * N, M * N};
            if (!tall) ti.push_back(TransItem{H + (int64_t)b * M * N, Y + (int64_t)b * M * N, M, N, M, N});
        }
        tick();
        launch_gen(h->kd, h->d_pts, h->d_nrm, h->d_tpad, meta(gi, cv), B, M, N, M * N, st);
        launch_sumsq(meta(si, cv), B, M * N, part, SUM_CHUNK, nrm, st);
        if (!tall) launch_transpose(meta(ti, cv), B, M * N, st);
        tock("s.gen");
        orthq(Y, rows, s, Q, R, qw, B, cv);
        // Jacobi input: R^T (tall) or R (wide)
        if (tall) {
            std::vector<TransItem> tr(B);
            for (int b = 0; b < B; ++b) tr[b] = TransItem{R + b * ss, A + b * ss, s, s, s, s};
            launch_transpose(meta(tr, cv), B, ss, st);
        } else {
            HIPCHK(hipMemcpyAsync(A, R, (size_t)B * ss * 8, hipMemcpyDeviceToDevice, st));
        }
        tock("s.qr");
        small_svd(A, J, S, B, s, cv);             // A <- W S, J <- rotations
        const double one = 1.0, zero = 0.0;
        const rocblas_operation NT = rocblas_operation_none;
        const rocblas_int ir = (rocblas_int)rows, is = s;
        // F = Q J (tall: U) or Q A (wide: V)
        RBCHK(rocblas_dgemm_strided_batched(rb, NT, NT, ir, is, is, &one, Q, ir, rows * s,
                                            tall ? J : A, is, ss, &zero, F, ir, rows * s, B));
        std::vector<RankItem> ri(B);
        for (int b = 0; b < B; ++b) {
            const Blk& k = h->blocks[idx[b]].b;
            RankItem r{};
            r.sigma = S + (int64_t)b * s;
            r.norm2p = nrm + b;
            r.extrap = nullptr;
            r.p = s;
            r.sketch = 0;
            r.pmin = (int)std::min(k.ie - k.ib, k.je - k.jb);
            ri[b] = r;
        }
        RankItem* dri = meta(ri, cv);
        launch_rank(dri, B, eps2, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpy(ri.data(), dri, B * sizeof(RankItem), hipMemcpyDeviceToHost));
        std::vector<int> ranks(B);
        for (int b = 0; b < B; ++b) {
            record_rank(idx[b], ri[b]);
            ranks[b] = ri[b].rank;
        }
        store_for(idx, ranks);
        std::vector<FinItem> fi;
        for (int b = 0; b < B; ++b) {
            const BlockRec& r = h->blocks[idx[b]];
            if (!ranks[b]) continue;
            FinItem f{};
            f.U = tall ? F + (int64_t)b * rows * s : J + b * ss;
            f.ldu = tall ? rows : s;
            f.V = tall ? A + b * ss : F + (int64_t)b * rows * s;
            f.ldv = tall ? s : rows;
            f.v_rows = 0;
            f.sigma = S + (int64_t)b * s;
            f.Uout = (double*)r.u_ptr;
            f.Vout = (double*)r.v_ptr;
            f.ib = r.b.ib;
            f.jb = r.b.jb;
            f.PI = r.PI;
            f.PJ = r.PJ;
            f.m = (int)(r.b.ie - r.b.ib);
            f.n = (int)(r.b.je - r.b.jb);
            f.k = ranks[b];
            fi.push_back(f);
        }
        if (!fi.empty()) launch_finalize(meta(fi, cv), (int)fi.size(), h->d_tpad, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipDeviceSynchronize());
        tock("s.rank+fin");
    }

    size_t exact_item_bytes(int64_t M, int64_t N) const {
        const int64_t rows = std::max(M, N), s = std::min(M, N);
        return 8 * (size_t)(2 * M * N + 2 * rows * s + 4 * s * s + s + 1 + (M * N) / SUM_CHUNK + 1 +
                            rows * s + 4 * s * s + 64 * s + s + jacobi_work(s) +
                            tall_work(rows, s)) + 16384;
    }
    // doubles of Jacobi workspace per item of width s
    static int64_t jacobi_work(int64_t s) {
        // the tiled Jacobi's copy of [A; J] and its preconditioning QR, or
        // rocSOLVER's three s x s buffers
        return s > 128 ? std::max<int64_t>(
                             s <= 512 ? 2 * s * jacobi_tiled_cols((int)s) + 9 * s * s + 70 * s : 0,
                             3 * s * s + 2 * s + 64)
                       : 0;
    }

    static bool verbose() {
        const char* v = getenv("HH_VERBOSE");
        return v && v[0] && v[0] != '0';
    }

    void check_info(const rocblas_int* dinfo, int B) {
        std::vector<rocblas_int> hi(B);
        HIPCHK(hipMemcpy(hi.data(), dinfo, B * sizeof(rocblas_int), hipMemcpyDeviceToHost));
        for (int b = 0; b < B; ++b)
            if (hi[b] != 0) fail(HH_EINTERNAL, "SVD did not converge (info " + std::to_string(hi[b]) + ")");
    }

    // Orthonormal basis of each rows x s item of Y (column-major, stride rows s):
    // Householder QR (geqrf) and the explicit Q = [I; 0] - V T V1^T with
    // T = (diag(1/tau) + striu(V^T V))^-1. Y is overwritten; R (s x s) optional.
    struct QrWork {
        double *tau, *Vm, *G, *Tinv, *T, *W, *W2, *W3;
    };
    QrWork qr_work(Carver& cv, int B, int64_t rows_max, int s) {
        QrWork w;
        w.W2 = cv.take<double>((size_t)B * 32 * s);
        w.W3 = cv.take<double>((size_t)B * 32 * s);
        w.tau = cv.take<double>((size_t)B * s);
        w.Vm = cv.take<double>((size_t)B * rows_max * s);
        w.G = cv.take<double>((size_t)B * s * s);
        w.Tinv = cv.take<double>((size_t)B * s * s);
        w.T = cv.take<double>((size_t)B * s * s);
        w.W = cv.take<double>((size_t)B * s * s);
        return w;
    }
    // Householder QR in place (geqrf layout). One kernel per item up to 4096
    // rows (or 64 columns); taller and wider matrices in 32-column panels whose
    // trailing columns are updated with the compact-WY form (I - V T V^T)^T
    // through batched GEMMs.
    void house_qr(double* Y, int64_t rows, int s, const QrWork& w, int B) {
        const int64_t strideA = rows * s;
        if (s <= 64 || rows <= 4096) {
            launch_house_qr(Y, rows, strideA, w.tau, s, rows, s, B, st);
            return;
        }
        const int nb = 32;
        const double one = 1.0, zero = 0.0, mone = -1.0;
        const int64_t nn = (int64_t)nb * nb;
        for (int p0 = 0; p0 < s; p0 += nb) {
            const int pw = std::min(nb, s - p0);
            const int64_t mp = rows - p0;
            double* panel = Y + (int64_t)p0 * rows + p0;
            launch_house_qr(panel, rows, strideA, w.tau + p0, s, mp, pw, B, st);
            const int rest = s - p0 - pw;
            if (rest <= 0) break;
            // V (mp x pw, in w.Vm), T (pw x pw, in w.T): T = (diag(1/tau) + striu(V^T V))^-1
            launch_panel_v(panel, rows, strideA, w.tau + p0, s, w.Vm, w.T, mp, pw, B, st);
            RBCHK(rocblas_dgemm_strided_batched(rb, rocblas_operation_transpose,
                                                rocblas_operation_none, pw, pw, (rocblas_int)mp,
                                                &one, w.Vm, (rocblas_int)mp, mp * pw, w.Vm,
                                                (rocblas_int)mp, mp * pw, &zero, w.G, pw, nn, B));
            launch_panel_tinv(w.G, w.tau + p0, s, w.Tinv, pw, B, st);
            RBCHK(rocblas_dtrsm_strided_batched(rb, rocblas_side_left, rocblas_fill_upper,
                                                rocblas_operation_none, rocblas_diagonal_non_unit,
                                                pw, pw, &one, w.Tinv, pw, nn, w.T, pw, nn, B));
            // C <- (I - V T V^T)^T C = C - V T^T (V^T C) for the trailing columns C
            double* C = panel + (int64_t)pw * rows;
            RBCHK(rocblas_dgemm_strided_batched(rb, rocblas_operation_transpose,
                                                rocblas_operation_none, pw, rest, (rocblas_int)mp,
                                                &one, w.Vm, (rocblas_int)mp, mp * pw, C,
                                                (rocblas_int)rows, strideA, &zero, w.W2, pw,
                                                (int64_t)pw * rest, B));
            RBCHK(rocblas_dgemm_strided_batched(rb, rocblas_operation_transpose,
                                                rocblas_operation_none, pw, rest, pw, &one, w.T,
                                                pw, nn, w.W2, pw, (int64_t)pw * rest, &zero, w.W3,
                                                pw, (int64_t)pw * rest, B));
            RBCHK(rocblas_dgemm_strided_batched(rb, rocblas_operation_none, rocblas_operation_none,
                                                (rocblas_int)mp, rest, pw, &mone, w.Vm,
                                                (rocblas_int)mp, mp * pw, w.W3, pw,
                                                (int64_t)pw * rest, &one, C, (rocblas_int)rows,
                                                strideA, B));
        }
    }

    void orthq(double* Y, int64_t rows, int s, double* Q, double* R, const QrWork& w, int B, Carver& cv) {
        if (rows > TSQR_CHUNK && s <= TSQR_CHUNK / 2) {
            orthq_tall(Y, rows, s, Q, R, B, cv);
            return;
        }
        const double one = 1.0, zero = 0.0, mone = -1.0;
        const rocblas_int ir = (rocblas_int)rows, is = s;
        const int64_t ss = (int64_t)s * s;
        tock("r.pre-orth");
        house_qr(Y, rows, s, w, B);
        tock(s <= 64 ? "q.house<=64" : "q.house>64");
        std::vector<QrItem> qi(B);
        for (int b = 0; b < B; ++b)
            qi[b] = QrItem{Y + b * rows * s, w.tau + (int64_t)b * s, w.Vm + b * rows * s,
                           R ? R + b * ss : nullptr, w.G + b * ss, w.Tinv + b * ss, w.T + b * ss,
                           Q + b * rows * s, rows};
        QrItem* dq = meta(qi, cv);
        launch_qr_extract(dq, B, rows, s, st);
        RBCHK(rocblas_dgemm_strided_batched(rb, rocblas_operation_transpose, rocblas_operation_none,
                                            is, is, ir, &one, w.Vm, ir, rows * s, w.Vm, ir, rows * s,
                                            &zero, w.G, is, ss, B));
        launch_qr_tinv(dq, B, s, st);
        RBCHK(rocblas_dtrsm_strided_batched(rb, rocblas_side_left, rocblas_fill_upper,
                                            rocblas_operation_none, rocblas_diagonal_non_unit, is, is,
                                            &one, w.Tinv, is, ss, w.T, is, ss, B));
        RBCHK(rocblas_dgemm_strided_batched(rb, rocblas_operation_none, rocblas_operation_transpose,
                                            is, is, is, &one, w.T, is, ss, w.Vm, ir, rows * s, &zero,
                                            w.W, is, ss, B));
        RBCHK(rocblas_dgemm_strided_batched(rb, rocblas_operation_none, rocblas_operation_none, ir,
                                            is, is, &mone, w.Vm, ir, rows * s, w.W, is, ss, &one, Q,
                                            ir, rows * s, B));
    }

    // Tall items (rows > TSQR_CHUNK): TSQR. The rows are cut into nch chunks of
    // at most TSQR_CHUNK rows (the last zero-padded: zero rows stay zero in Q),
    // each chunk is factored as above (one workgroup-sized kernel per chunk),
    // the chunks' s x s factors stacked ((nch s) x s per item) are factored
    // once more, and Q = diag(Q_c) Q_stack, i.e. chunk c of Q is Q_c times rows
    // c s .. c s + s - 1 of Q_stack; R is the stack's factor. The temporaries
    // are carved after the caller's buffers and released on return.
    void orthq_tall(double* Y, int64_t rows, int s, double* Q, double* R, int B, Carver& cv) {
        const size_t mark = cv.off;
        const int64_t nch = (rows + TSQR_CHUNK - 1) / TSQR_CHUNK;
        const int64_t ch = (rows + nch - 1) / nch;
        const int64_t ss = (int64_t)s * s;
        const int Bc = (int)(B * nch);
        double* C = cv.take<double>((size_t)Bc * ch * s);
        double* Qc = cv.take<double>((size_t)Bc * ch * s);
        double* Rc = cv.take<double>((size_t)Bc * ss);
        double* S = cv.take<double>((size_t)B * nch * ss);
        double* Qs = cv.take<double>((size_t)B * nch * ss);
        std::vector<CopyItem> ci(Bc), si(Bc);
        for (int b = 0; b < B; ++b)
            for (int64_t c = 0; c < nch; ++c) {
                const int64_t r0 = c * ch, m = std::min(ch, rows - r0), k = b * nch + c;
                ci[k] = CopyItem{Y + (int64_t)b * rows * s + r0, C + k * ch * s, m, s, rows, ch, ch};
                si[k] = CopyItem{Rc + k * ss, S + (int64_t)b * nch * ss + c * s, s, s, s, nch * s, s};
            }
        launch_copy2d(meta(ci, cv), Bc, ch * s, st);
        QrWork wc = qr_work(cv, Bc, ch, s);
        orthq(C, ch, s, Qc, Rc, wc, Bc, cv);
        launch_copy2d(meta(si, cv), Bc, ss, st);
        QrWork ws = qr_work(cv, B, nch * s, s);
        orthq(S, nch * s, s, Qs, R, ws, B, cv);
        const double one = 1.0, zero = 0.0;
        for (int64_t c = 0; c < nch; ++c) {
            const int64_t m = std::min(ch, rows - c * ch);
            RBCHK(rocblas_dgemm_strided_batched(
                rb, rocblas_operation_none, rocblas_operation_none, (rocblas_int)m, s, s, &one,
                Qc + c * ch * s, (rocblas_int)ch, nch * ch * s, Qs + c * s, (rocblas_int)(nch * s),
                nch * ss, &zero, Q + c * ch, (rocblas_int)rows, rows * s, B));
        }
        HIPCHK(hipGetLastError());
        cv.off = mark;
    }
    // Scratch doubles per item that orthq_tall adds for a rows x s item.
    static int64_t tall_work(int64_t rows, int64_t s) {
        if (rows <= TSQR_CHUNK || s > TSQR_CHUNK / 2) return 0;
        const int64_t nch = (rows + TSQR_CHUNK - 1) / TSQR_CHUNK;
        return 3 * (rows + nch) * s + 9 * nch * s * s + 4 * s * s + 70 * nch * s + 64;
    }

    // SVD of the s x s factors R (column-major, stride s^2): A <- U S, J <- V,
    // sigma decreasing. One-sided Jacobi up to 128 (in LDS up to 64, in
    // registers up to 128) and, for batches of at least JACOBI_TILED_MIN_BATCH
    // items, up to 512 (LDS tiles of a global copy: one workgroup per item, so
    // it pays only when the batch fills the GPU); otherwise rocSOLVER's SVD of
    // the square matrices (a non-converged item is retried alone in place
    // mode).
    void small_svd(double* R, double* J, double* S, int B, int s, Carver& cv) {
        const int64_t ss = (int64_t)s * s;
        std::vector<JacItem> ji(B);
        for (int b = 0; b < B; ++b) ji[b] = JacItem{R + b * ss, J + b * ss, S + (int64_t)b * s};
        JacItem* dj = meta(ji, cv);
        if (s <= 64) {
            launch_jacobi(dj, B, s, st);
            tock("c.jacobi");
            return;
        }
        if (s <= 128) {
            launch_jacobi128(dj, B, s, st);
            tock("c.jacobi128");
            return;
        }
        if (s <= 512 && B >= JACOBI_TILED_MIN_BATCH) {
            // Preconditioned: R^T = Q2 R2, then Jacobi on R2^T, whose sweeps
            // converge several times faster than on R itself (the rows of R2
            // are graded). R = R2^T Q2^T, so the Jacobi output A = R2^T J is
            // R's left vectors times S and R's right vectors are Q2 J.
            const size_t mark = cv.off;
            double* Rt = cv.take<double>((size_t)B * ss);
            double* Q2 = cv.take<double>((size_t)B * ss);
            double* R2 = cv.take<double>((size_t)B * ss);
            double* J2 = cv.take<double>((size_t)B * ss);
            std::vector<TransItem> t1(B), t2(B);
            std::vector<JacItem> jt(B);
            for (int b = 0; b < B; ++b) {
                t1[b] = TransItem{R + b * ss, Rt + b * ss, s, s, s, s};
                t2[b] = TransItem{R2 + b * ss, R + b * ss, s, s, s, s};
                jt[b] = JacItem{R + b * ss, J2 + b * ss, S + (int64_t)b * s};
            }
            launch_transpose(meta(t1, cv), B, ss, st);
            QrWork w = qr_work(cv, B, s, s);
            orthq(Rt, s, s, Q2, R2, w, B, cv);
            launch_transpose(meta(t2, cv), B, ss, st);
            double* work = cv.take<double>((size_t)B * 2 * s * jacobi_tiled_cols(s));
            launch_jacobi_tiled(meta(jt, cv), work, B, s, st);
            const double one = 1.0, zero = 0.0;
            RBCHK(rocblas_dgemm_strided_batched(rb, rocblas_operation_none, rocblas_operation_none,
                                                s, s, s, &one, Q2, s, ss, J2, s, ss, &zero, J, s,
                                                ss, B));
            HIPCHK(hipGetLastError());
            cv.off = mark;
            tock("c.jacobi512");
            return;
        }
        double* Rc = cv.take<double>((size_t)B * ss);
        double* Ug = cv.take<double>((size_t)B * ss);
        double* Vg = cv.take<double>((size_t)B * ss);
        double* Eg = cv.take<double>((size_t)B * s);
        rocblas_int* inf = cv.take<rocblas_int>(B);
        HIPCHK(hipMemcpy(Rc, R, (size_t)B * ss * 8, hipMemcpyDeviceToDevice));
        RBCHK(rocsolver_dgesvd_strided_batched(rb, rocblas_svect_singular, rocblas_svect_singular, s,
                                               s, Rc, s, ss, S, s, Ug, s, ss, Vg, s, ss, Eg, s,
                                               rocblas_outofplace, inf, B));
        std::vector<rocblas_int> hi(B);
        HIPCHK(hipMemcpy(hi.data(), inf, B * sizeof(rocblas_int), hipMemcpyDeviceToHost));
        for (int b = 0; b < B; ++b) {
            if (!hi[b]) continue;
            HIPCHK(hipMemcpy(Rc + b * ss, R + b * ss, ss * 8, hipMemcpyDeviceToDevice));
            RBCHK(rocsolver_dgesvd(rb, rocblas_svect_singular, rocblas_svect_singular, s, s,
                                   Rc + b * ss, s, S + (int64_t)b * s, Ug + b * ss, s, Vg + b * ss,
                                   s, Eg + (int64_t)b * s, rocblas_inplace, inf + b));
            rocblas_int v = 0;
            HIPCHK(hipMemcpy(&v, inf + b, sizeof(v), hipMemcpyDeviceToHost));
            if (v) fail(HH_EINTERNAL, "SVD of a sketch core did not converge");
        }
        launch_svd_to_jac(dj, Ug, Vg, B, s, st);
        tock("c.gesvd>64");
    }

    // One randomized round for a batch sharing sketch width s; returns the
    // blocks that need a wider sketch.
    std::vector<int64_t> random_batch(const std::vector<int64_t>& idx, int s, int round) {
        const int B = (int)idx.size();
        if (verbose()) {
            tsum["n.items s=" + std::to_string(s)] += B;
            tsum["n.batches s=" + std::to_string(s)] += 1;
        }
        int64_t M = 0, N = 0;
        for (int64_t i : idx) {
            M = std::max<int64_t>(M, h->blocks[i].b.ie - h->blocks[i].b.ib);
            N = std::max<int64_t>(N, h->blocks[i].b.je - h->blocks[i].b.jb);
        }
        const int64_t nch = (M * N + SUM_CHUNK - 1) / SUM_CHUNK;
        const int64_t ss = (int64_t)s * s;
        Carver cv{scratch, scratch_bytes};
        double* H = cv.take<double>((size_t)B * M * N);
        double* Om = cv.take<double>((size_t)B * N * s);
        double* Y = cv.take<double>((size_t)B * M * s);
        double* Q = cv.take<double>((size_t)B * M * s);
        double* Z = cv.take<double>((size_t)B * N * s);
        double* Q2 = cv.take<double>((size_t)B * N * s);
        double* R = cv.take<double>((size_t)B * ss);
        double* J = cv.take<double>((size_t)B * ss);
        double* S = cv.take<double>((size_t)B * s);
        double* nrm = cv.take<double>(B);
        double* e2 = cv.take<double>(B);
        double* part = cv.take<double>((size_t)B * nch);
        QrWork qw = qr_work(cv, B, std::max(M, N), s);
        std::vector<GenItem> gi(B);
        std::vector<SumItem> si(B);
        std::vector<SketchItem> ski(B);
        for (int b = 0; b < B; ++b) {
            const Blk& k = h->blocks[idx[b]].b;
            gi[b] = GenItem{k.ib, k.jb, k.ie - k.ib, k.je - k.jb, H + (int64_t)b * M * N, M, 0, 0};
            si[b] = SumItem{H + (int64_t)b * M * N, M * N};
            ski[b] = SketchItem{Om + (int64_t)b * N * s, k.je - k.jb, idx[b], round, 0};
        }
        tick();
        SumItem* dsi = meta(si, cv);
        launch_gen(h->kd, h->d_pts, h->d_nrm, h->d_tpad, meta(gi, cv), B, M, N, M * N, st);
        launch_sumsq(dsi, B, M * N, part, SUM_CHUNK, nrm, st);
        launch_sketch(meta(ski, cv), B, N, s, h->opt.seed, st);
        tock("r.gen");
        const double one = 1.0, zero = 0.0, mone = -1.0;
        const rocblas_operation NT = rocblas_operation_none, TR = rocblas_operation_transpose;
        const rocblas_int iM = (rocblas_int)M, iN = (rocblas_int)N, is = s;
        // range finder with one power iteration: Q = orth(H orth(H^T orth(H Omega)))
        RBCHK(rocblas_dgemm_strided_batched(rb, NT, NT, iM, is, iN, &one, H, iM, M * N, Om, iN,
                                            N * s, &zero, Y, iM, M * s, B));
        tock("r.gemm");
        orthq(Y, M, s, Q, nullptr, qw, B, cv);
        tock("r.orth");
        RBCHK(rocblas_dgemm_strided_batched(rb, TR, NT, iN, is, iM, &one, H, iM, M * N, Q, iM,
                                            M * s, &zero, Z, iN, N * s, B));
        tock("r.gemm");
        orthq(Z, N, s, Q2, nullptr, qw, B, cv);
        tock("r.orth");
        RBCHK(rocblas_dgemm_strided_batched(rb, NT, NT, iM, is, iN, &one, H, iM, M * N, Q2, iN,
                                            N * s, &zero, Y, iM, M * s, B));
        tock("r.gemm");
        orthq(Y, M, s, Q, nullptr, qw, B, cv);
        tock("r.orth");
        // B^T = H^T Q; H <- H - Q B and its Frobenius norm (the part Q misses)
        RBCHK(rocblas_dgemm_strided_batched(rb, TR, NT, iN, is, iM, &one, H, iM, M * N, Q, iM,
                                            M * s, &zero, Z, iN, N * s, B));
        RBCHK(rocblas_dgemm_strided_batched(rb, NT, TR, iM, iN, is, &mone, Q, iM, M * s, Z, iN,
                                            N * s, &one, H, iM, M * N, B));
        launch_sumsq(dsi, B, M * N, part, SUM_CHUNK, e2, st);
        tock("r.gemm");
        // SVD of B through B^T = Qb R: R = W S J^T gives B = J S (Qb W)^T
        orthq(Z, N, s, Q2, R, qw, B, cv);
        tock("r.orth");
        small_svd(R, J, S, B, s, cv);
        tock("r.coresvd");
        std::vector<RankItem> ri(B);
        for (int b = 0; b < B; ++b) {
            const Blk& k = h->blocks[idx[b]].b;
            RankItem r{};
            r.sigma = S + (int64_t)b * s;
            r.norm2p = nrm + b;
            r.extrap = e2 + b;
            r.p = s;
            r.sketch = s;
            r.pmin = (int)std::min(k.ie - k.ib, k.je - k.jb);
            r.oversample = OVERSAMPLE;
            ri[b] = r;
        }
        RankItem* dri = meta(ri, cv);
        launch_rank(dri, B, eps2, st);
        // U = Q J (M x s), V = Qb (W S) (N x s); only accepted items are kept
        RBCHK(rocblas_dgemm_strided_batched(rb, NT, NT, iM, is, is, &one, Q, iM, M * s, J, is, ss,
                                            &zero, Y, iM, M * s, B));
        RBCHK(rocblas_dgemm_strided_batched(rb, NT, NT, iN, is, is, &one, Q2, iN, N * s, R, is, ss,
                                            &zero, Z, iN, N * s, B));
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpy(ri.data(), dri, B * sizeof(RankItem), hipMemcpyDeviceToHost));
        std::vector<int64_t> acc_idx, retry;
        std::vector<int> acc_rank, acc_pos;
        for (int b = 0; b < B; ++b) {
            if (ri[b].accept) {
                record_rank(idx[b], ri[b]);
                acc_idx.push_back(idx[b]);
                acc_rank.push_back(ri[b].rank);
                acc_pos.push_back(b);
            } else {
                retry.push_back(idx[b]);
            }
        }
        if (!acc_idx.empty()) {
            store_for(acc_idx, acc_rank);
            std::vector<FinItem> fi;
            for (size_t a = 0; a < acc_idx.size(); ++a) {
                const BlockRec& r = h->blocks[acc_idx[a]];
                const int b = acc_pos[a];
                if (!acc_rank[a]) continue;
                FinItem f{};
                f.U = Y + (int64_t)b * M * s;
                f.V = Z + (int64_t)b * N * s;
                f.v_rows = 0;
                f.sigma = S + (int64_t)b * s;
                f.Uout = (double*)r.u_ptr;
                f.Vout = (double*)r.v_ptr;
                f.ib = r.b.ib;
                f.jb = r.b.jb;
                f.ldu = M;
                f.ldv = N;
                f.PI = r.PI;
                f.PJ = r.PJ;
                f.m = (int)(r.b.ie - r.b.ib);
                f.n = (int)(r.b.je - r.b.jb);
                f.k = acc_rank[a];
                fi.push_back(f);
            }
            if (!fi.empty()) launch_finalize(meta(fi, cv), (int)fi.size(), h->d_tpad, st);
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipDeviceSynchronize());
        tock("r.rank+fin");
        return retry;
    }

    size_t random_item_bytes(int64_t M, int64_t N, int64_t s) const {
        const int64_t mx = std::max(M, N);
        return 8 * (size_t)(M * N + 3 * N * s + 2 * M * s + mx * s + 6 * s * s + 64 * s + 4 * s + 3 +
                            (M * N) / SUM_CHUNK + 1 + jacobi_work(s) + tall_work(mx, s)) + 16384;
    }

    // Size bucket: dimensions within a factor 2^(1/4) share a bucket, so zero
    // padding to the batch maximum wastes at most ~19% per dimension.
    static int bucket(int64_t v) { return (int)std::ceil(4.0 * std::log2((double)std::max<int64_t>(v, 1))); }

    // Greedy batches of same-bucket blocks, bounded by the scratch budget.
    template <class F, class G>
    void batched(std::vector<int64_t> list, F item_bytes, G run) {
        auto key = [&](int64_t a) {
            const Blk& x = h->blocks[a].b;
            return std::make_pair(bucket(x.ie - x.ib), bucket(x.je - x.jb));
        };
        std::sort(list.begin(), list.end(), [&](int64_t a, int64_t b) {
            auto ka = key(a), kb = key(b);
            if (ka != kb) return ka > kb;
            return a < b;
        });
        size_t i = 0;
        const size_t budget = scratch_bytes * 9 / 10;
        while (i < list.size()) {
            std::vector<int64_t> batch;
            int64_t M = 0, N = 0;
            const auto k0 = key(list[i]);
            while (i < list.size() && batch.size() < 4096 && key(list[i]) == k0) {
                const Blk& k = h->blocks[list[i]].b;
                int64_t M2 = std::max<int64_t>(M, k.ie - k.ib), N2 = std::max<int64_t>(N, k.je - k.jb);
                if (!batch.empty() && item_bytes(M2, N2) * (batch.size() + 1) > budget) break;
                if (batch.empty() && item_bytes(M2, N2) > budget)
                    fail(HH_ENOMEM, "a single block does not fit the construction scratch");
                M = M2;
                N = N2;
                batch.push_back(list[i++]);
            }
            run(batch);
        }
    }

    void compress(const std::vector<int64_t>& cand) {
        std::vector<int64_t> exact, rnd;
        for (int64_t i : cand) {
            const Blk& k = h->blocks[i].b;
            (std::min(k.ie - k.ib, k.je - k.jb) <= EXACT_SVD_MAX ? exact : rnd).push_back(i);
        }
        total_cand = (int64_t)cand.size();
        batched(exact, [&](int64_t M, int64_t N) { return exact_item_bytes(M, N); },
                [&](const std::vector<int64_t>& b) {
                    exact_batch(b);
                    progress((int64_t)b.size(), "exact SVD");
                });
        // randomized: groups keyed by sketch width, widening on demand
        std::map<int, std::vector<int64_t>> queue;
        std::map<int64_t, int> rounds;
        for (int64_t i : rnd) {
            queue[SKETCH_START].push_back(i);
            rounds[i] = 0;
        }
        while (!queue.empty()) {
            auto it = queue.begin();
            const int s = it->first;
            std::vector<int64_t> list = std::move(it->second);
            queue.erase(it);
            // items with different round counters cannot share a launch (they do
            // share s, so rounds coincide unless s was clipped to min(m, n))
            std::map<int, std::vector<int64_t>> by_round;
            for (int64_t i : list) by_round[rounds[i]].push_back(i);
            for (auto& kv : by_round) {
                const int round = kv.first;
                batched(kv.second,
                        [&](int64_t M, int64_t N) { return random_item_bytes(M, N, s); },
                        [&](const std::vector<int64_t>& b) {
                            auto again = random_batch(b, s, round);
                            progress((int64_t)(b.size() - again.size()), "randomized");
                            for (int64_t r : again) {
                                const Blk& k = h->blocks[r].b;
                                int pmin = (int)std::min(k.ie - k.ib, k.je - k.jb);
                                int s2 = std::min(2 * s, pmin);
                                if (s2 <= s) fail(HH_EINTERNAL, "sketch cannot widen");
                                rounds[r] = round + 1;
                                queue[s2].push_back(r);
                            }
                        });
            }
        }
        progress(0, "done", true);
        report_times();
    }

    // Dense blocks generated in place (padded-row layout) and their norms.
    void dense(const std::vector<int64_t>& list) {
        if (list.empty()) return;
        int64_t total = 0;
        for (int64_t i : list) {
            const BlockRec& r = h->blocks[i];
            total += r.PI * (r.b.je - r.b.jb);
        }
        double* D = static_cast<double*>(h->mem.alloc((size_t)total * 8 + 256, true));
        int64_t off = 0;
        std::vector<GenItem> gi;
        std::vector<SumItem> si;
        int64_t maxmn = 0, maxcount = 0;
        for (int64_t i : list) {
            BlockRec& r = h->blocks[i];
            const int64_t m = r.b.ie - r.b.ib, n = r.b.je - r.b.jb;
            r.d_ptr = D + off;
            r.lowrank = false;
            r.rank = 0;
            r.fmt = HH_FMT_FP64;
            gi.push_back(GenItem{r.b.ib, r.b.jb, m, n, D + off, r.PI, 1, 0});
            si.push_back(SumItem{D + off, r.PI * n});
            maxmn = std::max(maxmn, m * n);
            maxcount = std::max(maxcount, r.PI * n);
            off += r.PI * n;
        }
        for (size_t a = 0; a < gi.size(); a += 32768) {
            size_t e = std::min(gi.size(), a + 32768);
            std::vector<GenItem> g(gi.begin() + a, gi.begin() + e);
            std::vector<SumItem> s(si.begin() + a, si.begin() + e);
            Carver cv{scratch, scratch_bytes};
            const int B = (int)g.size();
            const int64_t nch = (maxcount + SUM_CHUNK - 1) / SUM_CHUNK;
            double* part = cv.take<double>((size_t)B * nch);
            double* nrm = cv.take<double>(B);
            launch_gen(h->kd, h->d_pts, h->d_nrm, h->d_tpad, meta(g, cv), B, 0, 0, maxmn, st);
            launch_sumsq(meta(s, cv), B, maxcount, part, SUM_CHUNK, nrm, st);
            std::vector<double> hn(B);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpy(hn.data(), nrm, B * sizeof(double), hipMemcpyDeviceToHost));
            for (int b = 0; b < B; ++b) {
                BlockRec& r = h->blocks[list[a + b]];
                r.entry2 = hn[b];
                r.nb2 = hn[b];
            }
        }
    }

    // Alg. 3 storage: round every low-rank factor into its format's arena.
    void pack(bool in_place_ok = true) {
        int64_t need[NFMT_CODES] = {0, 0, 0, 0, 0, 0};   // bytes per format
        std::vector<int64_t> lr;
        for (size_t i = 0; i < h->blocks.size(); ++i) {
            const BlockRec& r = h->blocks[i];
            if (r.lowrank && r.rank > 0) {
                lr.push_back((int64_t)i);
                need[r.fmt] += (int64_t)r.rank * (col_bytes(r.fmt, r.t, r.PI) + col_bytes(r.fmt, r.t, r.PJ));
            }
        }
        bool all64 = need[1] == 0 && need[2] == 0 && need[3] == 0 && need[4] == 0 && need[5] == 0;
        h->all_fp64 = all64;
        h->has_cont = need[HH_FMT_CONT] > 0;
        h->family = h->has_cont ? FAM_CONT : need[HH_FMT_Q43] > 0 ? FAM_Q43 : FAM_FIX;
        if (all64 && in_place_ok) {
            // The fp64 store can serve as the arena as it is; it is re-laid in
            // cluster order (longer runs in the product) only if a second copy
            // fits in free device memory with 4 GiB to spare.
            size_t fr = 0, tot = 0;
            HIPCHK(hipMemGetInfo(&fr, &tot));
            if ((double)fr < (double)need[0] + (double)(4ull << 30)) return;
        }
        // exponents of the scaled formats (fp16, bf16, q43)
        std::vector<double> mx(2 * lr.size(), 0.0);
        {
            std::vector<SumItem> items;
            for (int64_t i : lr) {
                const BlockRec& r = h->blocks[i];
                items.push_back(SumItem{(const double*)r.u_ptr, (int64_t)r.rank * r.PI});
                items.push_back(SumItem{(const double*)r.v_ptr, (int64_t)r.rank * r.PJ});
            }
            for (size_t a = 0; a < items.size(); a += 65536) {
                size_t e = std::min(items.size(), a + 65536);
                std::vector<SumItem> part(items.begin() + a, items.begin() + e);
                Carver cv{scratch, scratch_bytes};
                double* out = cv.take<double>(part.size());
                launch_maxabs(meta(part, cv), (int)part.size(), out, st);
                HIPCHK(hipGetLastError());
                HIPCHK(hipMemcpy(mx.data() + a, out, part.size() * 8, hipMemcpyDeviceToHost));
            }
        }
        char* arena[NFMT_CODES] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        for (int f = 0; f < NFMT_CODES; ++f)
            if (need[f]) arena[f] = static_cast<char*>(h->mem.alloc((size_t)need[f] + 256, false));
        // Arena of a format: every U in (level, row box, column box) order, then
        // every V in (level, column box, row box) order, so that the factors
        // of one cluster and format follow each other (one strided matrix).
        int64_t offU[NFMT_CODES] = {0, 0, 0, 0, 0, 0}, offV[NFMT_CODES] = {0, 0, 0, 0, 0, 0};
        for (int64_t i : lr) {
            const BlockRec& r = h->blocks[i];
            offV[r.fmt] += (int64_t)r.rank * col_bytes(r.fmt, r.t, r.PI);
        }
        std::vector<int64_t> lr_t(lr);
        std::stable_sort(lr_t.begin(), lr_t.end(), [&](int64_t x, int64_t y) {
            const Blk &a = h->blocks[x].b, &b = h->blocks[y].b;
            return std::make_tuple(a.level, a.bj, a.bi) < std::make_tuple(b.level, b.bj, b.bi);
        });
        for (size_t a = 0; a < lr.size(); ++a) {
            BlockRec& r = h->blocks[lr[a]];
            auto expo = [&](double m) {
                if ((r.fmt != HH_FMT_FP16 && r.fmt != HH_FMT_BF16 && r.fmt != HH_FMT_Q43) ||
                    m == 0.0)
                    return 0;
                int q;
                std::frexp(m, &q);
                // largest entry scaled into [2^14, 2^15) (fp16), [1, 2) (bf16), [64, 128) (q43)
                return r.fmt == HH_FMT_FP16 ? q - 1 - 14 : r.fmt == HH_FMT_Q43 ? q - 1 - 6 : q - 1;
            };
            r.eU = expo(mx[2 * a]);
            r.eV = expo(mx[2 * a + 1]);
        }
        std::vector<PackItem> items;
        std::vector<ContPackItem> citems;
        int64_t maxcount = 0, maxdw = 0;
        auto add = [&](const BlockRec& r, const void* src, char* dst, int64_t P, int e) {
            if (r.fmt == HH_FMT_CONT) {
                const int64_t cdw = col_bytes(r.fmt, r.t, P) / 4;
                citems.push_back(ContPackItem{(const double*)src, reinterpret_cast<uint32_t*>(dst), P,
                                              cdw, r.rank, r.t});
                maxdw = std::max(maxdw, (int64_t)r.rank * cdw);
            } else {
                items.push_back(PackItem{(const double*)src, dst, (int64_t)r.rank * P, r.fmt, e});
                maxcount = std::max(maxcount, (int64_t)r.rank * P);
            }
        };
        std::vector<const void*> newU(h->blocks.size(), nullptr), newV(h->blocks.size(), nullptr);
        for (int64_t i : lr) {
            BlockRec& r = h->blocks[i];
            char* up = arena[r.fmt] + offU[r.fmt];
            offU[r.fmt] += (int64_t)r.rank * col_bytes(r.fmt, r.t, r.PI);
            add(r, r.u_ptr, up, r.PI, r.eU);
            newU[i] = up;
        }
        for (int64_t i : lr_t) {
            BlockRec& r = h->blocks[i];
            char* vp = arena[r.fmt] + offV[r.fmt];
            offV[r.fmt] += (int64_t)r.rank * col_bytes(r.fmt, r.t, r.PJ);
            add(r, r.v_ptr, vp, r.PJ, r.eV);
            newV[i] = vp;
        }
        for (int64_t i : lr) {
            h->blocks[i].u_ptr = newU[i];
            h->blocks[i].v_ptr = newV[i];
        }
        for (size_t a = 0; a < items.size(); a += 32768) {
            size_t e = std::min(items.size(), a + 32768);
            std::vector<PackItem> part(items.begin() + a, items.begin() + e);
            Carver cv{scratch, scratch_bytes};
            launch_pack(meta(part, cv), (int)part.size(), maxcount, st);
            HIPCHK(hipGetLastError());
            HIPCHK(hipDeviceSynchronize());
        }
        for (size_t a = 0; a < citems.size(); a += 32768) {
            size_t e = std::min(citems.size(), a + 32768);
            std::vector<ContPackItem> part(citems.begin() + a, citems.begin() + e);
            Carver cv{scratch, scratch_bytes};
            launch_pack_cont(meta(part, cv), (int)part.size(), maxdw, st);
            HIPCHK(hipGetLastError());
            HIPCHK(hipDeviceSynchronize());
        }
        store.free_all();
    }
};

// ----------------------------------------------------------- layout + tasks
static void layout(hh_handle* h) {
    const Plan& P = h->plan;
    const int L = P.L, d = P.d;
    const auto& rl = P.ranges[L];
    const int64_t nleaf = (int64_t)1 << (d * L);
    h->leaf_poff.assign(nleaf, 0);
    h->leaf_psz.assign(nleaf, 0);
    h->tpad.assign(P.n, 0);
    int64_t off = 0;
    for (int64_t b = 0; b < nleaf; ++b) {
        int64_t cnt = rl[2 * b + 1] - rl[2 * b];
        h->leaf_poff[b] = off;
        h->leaf_psz[b] = (cnt + ROW_PAD - 1) / ROW_PAD * ROW_PAD;
        for (int64_t t = rl[2 * b]; t < rl[2 * b + 1]; ++t) h->tpad[t] = off + (t - rl[2 * b]);
        off += h->leaf_psz[b];
    }
    h->np = off;
    auto cluster = [&](int level, int64_t box, int64_t& start, int64_t& len) {
        int sh = d * (L - level);
        int64_t first = box << sh, last = ((box + 1) << sh) - 1;
        start = h->leaf_poff[first];
        len = h->leaf_poff[last] + h->leaf_psz[last] - start;
    };
    h->blocks.resize(P.blocks.size());
    for (size_t i = 0; i < P.blocks.size(); ++i) {
        BlockRec& r = h->blocks[i];
        r = BlockRec{};
        r.b = P.blocks[i];
        cluster(r.b.level, r.b.bi, r.pI, r.PI);
        cluster(r.b.level, r.b.bj, r.pJ, r.PJ);
    }
}

// Blocks grouped for one direction of the product: by (level, row box) for
// H, by (level, column box) for H^T, each group in storage-format order
// (fp64, fp32, fp16, bf16) and then by the other box index. Factor arenas and
// coefficient indices follow these orders, so the blocks of one group and
// format are one strided matrix with consecutive coefficients.
static std::vector<int64_t> direction_order(const hh_handle* h, bool trans) {
    std::vector<int64_t> idx;
    for (size_t i = 0; i < h->blocks.size(); ++i) idx.push_back((int64_t)i);
    auto key = [&](int64_t i) {
        const BlockRec& r = h->blocks[i];
        const int f = r.lowrank ? r.fmt : HH_FMT_FP64;
        return trans ? std::make_tuple(r.b.level, r.b.bj, f, r.b.bi)
                     : std::make_tuple(r.b.level, r.b.bi, f, r.b.bj);
    };
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return key(x) < key(y); });
    return idx;
}

// Bytes between consecutive columns of a run, and of one column's slice of P
// rows (continuum entries are w bits).
static int64_t run_col_bytes(const Run& rn) {
    return rn.fmt == HH_FMT_CONT ? (int64_t)rn.stride * 4 : (int64_t)rn.stride * (int64_t)fmt_size(rn.fmt);
}
static int64_t slice_bytes(const Run& rn, int64_t P) {
    return rn.fmt == HH_FMT_CONT ? (P * rn.w + 7) / 8 : P * (int64_t)fmt_size(rn.fmt);
}

// Partial-row buffer of the work units, grown to the current tables' need.
static void ensure_part(hh_handle* h) {
    if (h->part && h->part_rows <= h->part_cap) return;
    const int64_t rows = std::max<int64_t>(h->part_rows, 1);
    double* p = static_cast<double*>(h->mem.alloc((size_t)rows * 8 + 256, true));
    if (h->part) h->mem.release(h->part);
    h->part = p;
    h->part_cap = rows;
}

// Frees the device copies of a direction's task tables (before a rebuild).
static void drop_tasks(hh_handle* h, TaskSet& S) {
    for (void* p : {(void*)S.d_dot, (void*)S.d_dotm, (void*)S.d_dotp, (void*)S.d_dot1p, (void*)S.d_pcols,
                    (void*)S.d_leaf, (void*)S.d_runs, (void*)S.d_cl_run, (void*)S.d_unit,
                    (void*)S.d_uruns, (void*)S.d_fin})
        if (p) h->mem.release(p);
    S = TaskSet{};
}

static void build_tasks(hh_handle* h) {
    const Plan& P = h->plan;
    const int L = P.L, d = P.d;
    const int64_t UNIT_BYTES = h->unit_bytes > 0 ? h->unit_bytes : hh::UNIT_BYTES;
    const int64_t DOT_TASK_ELEMS = h->dot_task_elems > 0 ? h->dot_task_elems : hh::DOT_TASK_ELEMS;
    drop_tasks(h, h->fwd);
    drop_tasks(h, h->bwd);
    h->part_rows = 0;
    const std::vector<int64_t> ord_f = direction_order(h, false), ord_t = direction_order(h, true);
    int64_t col = 0, col_t = 0;
    for (int64_t i : ord_f) {
        BlockRec& r = h->blocks[i];
        if (r.lowrank && r.rank > 0) {
            r.col = col;
            col += r.rank;
        }
    }
    for (int64_t i : ord_t) {
        BlockRec& r = h->blocks[i];
        if (r.lowrank && r.rank > 0) {
            r.col_t = col_t;
            col_t += r.rank;
        }
    }
    h->ncols = col;
    TaskSet& F = h->fwd;
    TaskSet& T = h->bwd;
    if (h->np >= ((int64_t)1 << 31) || h->ncols >= ((int64_t)1 << 31))
        fail(HH_ENOTSUP, "padded length and stored columns must stay below 2^31");
    // phase V tasks: the forward product dots V with x_J into tb[col], the
    // transpose dots U with x_I into tb[col_t]; the factor scales go into tb
    for (const auto& r : h->blocks) {
        if (!(r.lowrank && r.rank > 0)) continue;
        const int wbits = r.fmt == HH_FMT_CONT ? 9 + r.t : 0;
        for (int pass = 0; pass < 2; ++pass) {
            const int64_t Pl = pass == 0 ? r.PJ : r.PI;
            const int64_t cbytes = col_bytes(r.fmt, r.t, Pl);
            const char* base = static_cast<const char*>(pass == 0 ? r.v_ptr : r.u_ptr);
            // about DOT_TASK_ELEMS elements per task and at least one column per
            // wave; columns too long for the LDS stage of x go four to a wave
            const int64_t cmin = Pl > DOT_X_LDS ? 16 : 4;
            const int64_t cpt = std::min<int64_t>(
                r.rank, std::max<int64_t>(cmin, DOT_TASK_ELEMS / std::max<int64_t>(Pl, 1)));
            for (int64_t c0 = 0; c0 < r.rank; c0 += cpt) {
                DotTask t{};
                t.col0 = base + (size_t)(c0 * cbytes);
                t.xoff = pass == 0 ? r.pJ : r.pI;
                t.toff = (pass == 0 ? r.col : r.col_t) + c0;
                t.P = (int32_t)Pl;
                t.ncols = (int32_t)std::min<int64_t>(cpt, r.rank - c0);
                t.fmt = r.fmt;
                t.hid = 0;
                t.exp = r.eU + r.eV + fmt_exp_bias(r.fmt);
                t.w = wbits;
                (pass == 0 ? F : T).dot.push_back(t);
            }
            for (int64_t c0 = 0; c0 < r.rank; c0 += 16 * DOTM_MT) {
                DotTask t{};
                t.col0 = base + (size_t)(c0 * cbytes);
                t.xoff = pass == 0 ? r.pJ : r.pI;
                t.toff = (pass == 0 ? r.col : r.col_t) + c0;
                t.P = (int32_t)Pl;
                t.ncols = (int32_t)std::min<int64_t>(16 * DOTM_MT, r.rank - c0);
                t.fmt = r.fmt;
                t.hid = 0;
                t.exp = r.eU + r.eV + fmt_exp_bias(r.fmt);
                t.w = wbits;
                (pass == 0 ? F : T).dotm.push_back(t);
            }
        }
    }
    // clusters in (level, box) order; cluster (l, b) has index
    // sum_{l' < l} 2^(d l') + b
    std::vector<int64_t> first(L + 2, 0);
    for (int l = 0; l <= L; ++l) first[l + 1] = first[l] + ((int64_t)1 << (d * l));
    const int64_t ncl = first[L + 1];
    const int64_t nleaf = (int64_t)1 << (d * L);
    // transposed copies of the dense blocks: the product with H^T applies them
    // as ordinary runs of the column cluster (made once; a rebuild of the
    // tables keeps them)
    bool have_t = false;
    for (const auto& r : h->blocks)
        if (!r.lowrank) {
            have_t = r.dt_ptr != nullptr;
            break;
        }
    if (!have_t) {
        int64_t total = 0;
        for (const auto& r : h->blocks)
            if (!r.lowrank) total += r.PJ * (r.b.ie - r.b.ib);
        double* DT = static_cast<double*>(h->mem.alloc((size_t)std::max<int64_t>(total, 1) * 8 + 256, true));
        std::vector<TransItem> items;
        int64_t off = 0, maxcount = 0;
        for (auto& r : h->blocks) {
            if (r.lowrank) continue;
            const int64_t m = r.b.ie - r.b.ib, n = r.b.je - r.b.jb;
            r.dt_ptr = DT + off;
            items.push_back(TransItem{r.d_ptr, DT + off, m, n, r.PI, r.PJ});
            maxcount = std::max(maxcount, m * n);
            off += r.PJ * m;
        }
        for (size_t a = 0; a < items.size(); a += 32768) {
            const size_t e = std::min(items.size(), a + 32768);
            std::vector<TransItem> part(items.begin() + a, items.begin() + e);
            DevMem tmp;
            TransItem* d_items = upload(tmp, part);
            launch_transpose(d_items, (int)part.size(), maxcount, nullptr);
            HIPCHK(hipGetLastError());
            HIPCHK(hipDeviceSynchronize());
        }
    }
    const int64_t run_lim = run_bytes_max();
    for (int dir = 0; dir < 2; ++dir) {
        TaskSet& S = dir == 0 ? F : T;
        const std::vector<int64_t>& ord = dir == 0 ? ord_f : ord_t;
        std::vector<std::vector<Run>> per(ncl);
        for (int64_t bi : ord) {
            const BlockRec& r = h->blocks[bi];
            const int64_t box = dir == 0 ? r.b.bi : r.b.bj;
            const int64_t ci = first[r.b.level] + box;
            Run rn{};
            if (r.lowrank) {
                if (r.rank == 0) continue;
                rn.base = dir == 0 ? r.u_ptr : r.v_ptr;
                rn.pc = dir == 0 ? r.pI : r.pJ;
                // stride in elements; for continuum columns in dwords
                rn.stride = (int32_t)(r.fmt == HH_FMT_CONT ? col_bytes(r.fmt, r.t, dir == 0 ? r.PI : r.PJ) / 4
                                                           : (dir == 0 ? r.PI : r.PJ));
                rn.toff = (int32_t)(dir == 0 ? r.col : r.col_t);
                rn.ncols = r.rank;
                rn.fmt = (int8_t)r.fmt;
                rn.w = (int16_t)(r.fmt == HH_FMT_CONT ? 9 + r.t : 0);
                rn.from_x = 0;
            } else if (dir == 0) {
                rn.base = r.d_ptr;
                rn.pc = r.pI;
                rn.stride = (int32_t)r.PI;
                rn.toff = (int32_t)r.pJ;
                rn.ncols = (int32_t)(r.b.je - r.b.jb);
                rn.fmt = HH_FMT_FP64;
                rn.from_x = 1;
            } else {
                rn.base = r.dt_ptr;
                rn.pc = r.pJ;
                rn.stride = (int32_t)r.PJ;
                rn.toff = (int32_t)r.pI;
                rn.ncols = (int32_t)(r.b.ie - r.b.ib);
                rn.fmt = HH_FMT_FP64;
                rn.from_x = 1;
            }
            // merge with the previous run when the columns continue it and the
            // merged run stays under the buffer-offset limit
            std::vector<Run>& lst = per[ci];
            const int64_t cb = run_col_bytes(rn);                                // bytes per column
            if (cb > run_lim)
                fail(HH_ENOTSUP, "a factor column spans more bytes than one buffer descriptor addresses");
            const int64_t cmax = run_lim / cb;
            if (!lst.empty() && !rn.from_x) {
                Run& pr = lst.back();
                const char* end = static_cast<const char*>(pr.base) + (size_t)pr.ncols * run_col_bytes(pr);
                if (!pr.from_x && pr.fmt == rn.fmt && pr.w == rn.w && pr.stride == rn.stride && pr.pc == rn.pc &&
                    end == rn.base && pr.toff + pr.ncols == rn.toff &&
                    (int64_t)pr.ncols + rn.ncols <= cmax) {
                    pr.ncols += rn.ncols;
                    continue;
                }
            }
            for (int64_t c0 = 0; c0 < rn.ncols; c0 += cmax) {
                Run piece = rn;
                piece.base = static_cast<const char*>(rn.base) + (size_t)(c0 * cb);
                piece.toff = rn.toff + (int32_t)c0;
                piece.ncols = (int32_t)std::min<int64_t>(cmax, rn.ncols - c0);
                lst.push_back(piece);
            }
        }
        // within a cluster, runs grouped by format slot (fp64, fp32, fp16,
        // bf16, continuum or q43)
        S.cl_run.assign(NFMT * ncl + 1, 0);
        for (int64_t c = 0; c < ncl; ++c)
            for (int f = 0; f < NFMT; ++f) {
                S.cl_run[NFMT * c + f] = (int32_t)S.runs.size();
                for (const Run& rn : per[c])
                    if (fmt_slot(rn.fmt) == f) S.runs.push_back(rn);
            }
        S.cl_run[NFMT * ncl] = (int32_t)S.runs.size();
        for (int64_t lf = 0; lf < nleaf; ++lf) {
            if (h->leaf_psz[lf] == 0) continue;
            LeafTask lt{};
            lt.poff = h->leaf_poff[lf];
            lt.P = (int32_t)h->leaf_psz[lf];
            lt.leaf = (int32_t)lf;
            lt.hid = 0;
            S.leaf.push_back(lt);
        }
        // single-vector work units: each leaf's runs in (format, level) order,
        // cut into slices of about UNIT_BYTES of factor data (long runs are
        // split by columns)
        int64_t po = 0;
        std::vector<std::vector<UnitTask>> by_leaf;
        for (const LeafTask& lt : S.leaf) {
            FinishTask ft{};
            ft.poff = lt.poff;
            ft.po = po;
            ft.P = lt.P;
            ft.leaf = lt.leaf;
            ft.hid = 0;
            std::vector<Run> list;                   // pieces in processing order
            for (int f = 0; f < NFMT; ++f)
                for (int l = 0; l <= L; ++l) {
                    const int64_t ci = first[l] + ((int64_t)lt.leaf >> (d * (L - l)));
                    for (const Run& rn : per[ci]) {
                        if (fmt_slot(rn.fmt) != f) continue;
                        const int64_t colb = std::max<int64_t>(
                            1, std::min<int64_t>(UNIT_BYTES / std::max<int64_t>(slice_bytes(rn, lt.P), 1),
                                                 run_lim / run_col_bytes(rn)));
                        for (int32_t c0 = 0; c0 < rn.ncols; c0 += (int32_t)colb) {
                            Run sub = rn;
                            sub.base = static_cast<const char*>(rn.base) + (size_t)c0 * run_col_bytes(rn);
                            sub.toff = rn.toff + c0;
                            sub.ncols = (int32_t)std::min<int64_t>(colb, rn.ncols - c0);
                            list.push_back(sub);
                        }
                    }
                }
            std::vector<UnitTask> units;
            size_t a = 0;
            while (a < list.size()) {
                size_t e = a;
                int64_t bytes = 0;
                while (e < list.size() && bytes < UNIT_BYTES) {
                    const int64_t b = (int64_t)list[e].ncols * slice_bytes(list[e], lt.P);
                    if (e > a && bytes + b > UNIT_BYTES + UNIT_BYTES / 2) break;
                    bytes += b;
                    ++e;
                }
                UnitTask ut{};
                ut.poff = lt.poff;
                ut.po = po;
                ut.P = lt.P;
                ut.rb = (int32_t)S.uruns.size();
                for (int f = 0; f < NFMT; ++f) {
                    for (size_t i = a; i < e; ++i)
                        if (fmt_slot(list[i].fmt) == f) S.uruns.push_back(list[i]);
                    ut.fe[f] = (int32_t)S.uruns.size();
                }
                ut.hid = 0;
                units.push_back(ut);
                po += lt.P;
                ft.nu++;
                a = e;
            }
            by_leaf.push_back(units);
            S.fin.push_back(ft);
        }
        h->part_rows = std::max(h->part_rows, po);
        // dispatch order: unit k of every leaf (Morton order), then unit k + 1,
        // so that waves running together read neighbouring rows of the same runs
        for (size_t k = 0;; ++k) {
            bool any = false;
            for (const auto& units : by_leaf)
                if (k < units.size()) {
                    S.unit.push_back(units[k]);
                    any = true;
                }
            if (!any) break;
        }
    }
    // several-RHS accumulation: one workgroup per leaf, so leaves go heaviest
    // first (their factor bytes), which shortens the tail of the launch; the
    // single-vector work units keep their own order
    for (TaskSet* S : {&F, &T}) {
        std::vector<std::pair<double, LeafTask>> wl;
        for (const LeafTask& lt : S->leaf) {
            double w = 0.0;
            for (int l = 0; l <= L; ++l) {
                const int64_t ci = first[l] + ((int64_t)lt.leaf >> (d * (L - l)));
                for (int32_t k = S->cl_run[NFMT * ci]; k < S->cl_run[NFMT * ci + NFMT]; ++k) {
                    const Run& rn = S->runs[k];
                    w += (double)rn.ncols * (rn.fmt == HH_FMT_CONT ? rn.w / 8.0 : fmt_size(rn.fmt));
                }
            }
            wl.push_back({w * lt.P, lt});
        }
        std::stable_sort(wl.begin(), wl.end(),
                         [](const auto& a, const auto& b) { return a.first > b.first; });
        for (size_t k = 0; k < wl.size(); ++k) S->leaf[k] = wl[k].second;
    }
    // panel tiles: the factors that phase V reads (V for H, U for H^T) in
    // memory order; blocks stored one after another with the same format,
    // entry width, stride and x slice form a panel, cut into tiles of
    // 16 DOTP_MT columns that may span blocks
    for (int dir = 0; dir < 2; ++dir) {
        TaskSet& S = dir == 0 ? F : T;
        std::vector<int64_t> lr;
        for (size_t i = 0; i < h->blocks.size(); ++i)
            if (h->blocks[i].lowrank && h->blocks[i].rank > 0) lr.push_back((int64_t)i);
        auto fptr = [&](int64_t i) {
            const BlockRec& r = h->blocks[i];
            return static_cast<const char*>(dir == 0 ? r.v_ptr : r.u_ptr);
        };
        std::sort(lr.begin(), lr.end(), [&](int64_t a, int64_t b) { return fptr(a) < fptr(b); });
        size_t g0 = 0;
        while (g0 < lr.size()) {
            const BlockRec& r0 = h->blocks[lr[g0]];
            const int64_t Pl = dir == 0 ? r0.PJ : r0.PI, xo = dir == 0 ? r0.pJ : r0.pI;
            const int64_t cbytes = col_bytes(r0.fmt, r0.t, Pl);
            // the panel: following blocks that continue it in memory
            size_t g1 = g0 + 1;
            const char* next = fptr(lr[g0]) + r0.rank * cbytes;
            while (g1 < lr.size()) {
                const BlockRec& r = h->blocks[lr[g1]];
                const int64_t P2 = dir == 0 ? r.PJ : r.PI, x2 = dir == 0 ? r.pJ : r.pI;
                if (r.fmt != r0.fmt || r.t != r0.t || P2 != Pl || x2 != xo || fptr(lr[g1]) != next) break;
                next += r.rank * cbytes;
                ++g1;
            }
            const int64_t m0 = (int64_t)S.pcols.size();
            for (size_t g = g0; g < g1; ++g) {
                const BlockRec& r = h->blocks[lr[g]];
                const int64_t base = dir == 0 ? r.col : r.col_t;
                const int64_t ex = r.eU + r.eV + fmt_exp_bias(r.fmt) + 1024;
                for (int64_t j = 0; j < r.rank; ++j) S.pcols.push_back((base + j) | (ex << 40));
            }
            const int64_t ncols = (int64_t)S.pcols.size() - m0;
            for (int64_t c0 = 0; c0 < ncols; c0 += 16 * DOTP_MT) {
                DotTask t{};
                t.col0 = fptr(lr[g0]) + c0 * cbytes;
                t.xoff = xo;
                t.toff = m0 + c0;                    // map position until the upload
                t.P = (int32_t)Pl;
                t.ncols = (int32_t)std::min<int64_t>(16 * DOTP_MT, ncols - c0);
                t.fmt = r0.fmt;
                t.hid = 0;
                t.exp = 0;
                t.w = r0.fmt == HH_FMT_CONT ? 9 + r0.t : 0;
                S.dotp.push_back(t);
            }
            // one right-hand side: about DOT_TASK_ELEMS elements per panel
            // task, at least 16 DOTP_MT columns
            if (r0.fmt != HH_FMT_CONT) {
                const int64_t cpt = std::max<int64_t>(16 * DOTP_MT, DOT_TASK_ELEMS / std::max<int64_t>(Pl, 1));
                for (int64_t c0 = 0; c0 < ncols; c0 += cpt) {
                    DotTask t{};
                    t.col0 = fptr(lr[g0]) + c0 * cbytes;
                    t.xoff = xo;
                    t.toff = m0 + c0;                // map position until the upload
                    t.P = (int32_t)Pl;
                    t.ncols = (int32_t)std::min<int64_t>(cpt, ncols - c0);
                    t.fmt = r0.fmt;
                    t.hid = 0;
                    t.exp = 0;
                    t.w = 0;
                    S.dot1p.push_back(t);
                }
            }
            g0 = g1;
        }
    }
    // several-RHS tiles ordered by the cluster of x they read (column cluster
    // for H, row cluster for H^T), so that x_J stays in L2 across its blocks
    for (int dir = 0; dir < 2; ++dir) {
        for (std::vector<DotTask>* v : {&(dir == 0 ? F : T).dotm, &(dir == 0 ? F : T).dotp,
                                        &(dir == 0 ? F : T).dot1p})
            std::stable_sort(v->begin(), v->end(), [](const DotTask& a, const DotTask& b) {
                return std::make_tuple(a.P, a.xoff) < std::make_tuple(b.P, b.xoff);
            });
    }
    for (TaskSet* S : {&F, &T}) {
        S->d_pcols = upload(h->mem, S->pcols);
        for (std::vector<DotTask>* v : {&S->dotp, &S->dot1p})
            for (DotTask& t : *v) {
                t.cmap = S->d_pcols + t.toff;
                t.toff = 0;
            }
        double dot_bytes = 0.0;
        for (const DotTask& t : S->dot) dot_bytes += (double)t.ncols * t.P * (double)fmt_size(t.fmt);
        S->dot_panel = !h->has_cont && !S->dot.empty() && 2 * S->dot1p.size() <= S->dot.size() &&
                       dot_bytes < (double)DOT_PANEL_BELOW * (double)S->dot.size();
        if (!S->dot_panel) S->dot1p.clear();
        S->d_dot = upload(h->mem, S->dot);
        S->d_dotm = upload(h->mem, S->dotm);
        S->d_dotp = upload(h->mem, S->dotp);
        S->d_dot1p = upload(h->mem, S->dot1p);
        S->d_leaf = upload(h->mem, S->leaf);
        S->d_runs = upload(h->mem, S->runs);
        S->d_cl_run = upload(h->mem, S->cl_run);
        S->d_unit = upload(h->mem, S->unit);
        S->d_uruns = upload(h->mem, S->uruns);
        S->d_fin = upload(h->mem, S->fin);
    }
}

// Alg. 3 (eq:amp_prec_choice, evaluated squared: u^2 2^(d l) ||H~_b||^2 <=
// eps^2 ||H~||^2, ties pass): the lowest precision of the mask that passes,
// else fp64. With continuum storage (the accessor remark of Sec. 4.3) the
// candidates are t = 7..23 fraction bits with u = 2^-(t + 1), smallest t first.
static void choose_lowrank_format(const BlockRec& r, double total2, int d, double eps,
                                  const hh_options& o, int& fmt, int& t) {
    const double rhs = (eps * eps) * total2;
    const double lhs = std::ldexp(1.0, d * r.b.level) * r.nb2;
    t = 0;
    if (o.continuum) {
        // continuum = 2: only the byte-aligned widths 16, 24, 32 (t = 7, 15, 23)
        const int step = o.continuum == 2 ? 8 : 1;
        for (int tt = 7; tt <= 23; tt += step) {
            const double u = std::ldexp(1.0, -(tt + 1));
            if ((u * u) * lhs <= rhs) {
                fmt = HH_FMT_CONT;
                t = tt;
                return;
            }
        }
        fmt = HH_FMT_FP64;
        return;
    }
    const int order[4] = {HH_FMT_Q43, HH_FMT_BF16, HH_FMT_FP16, HH_FMT_FP32};
    for (int f : order) {
        if (!(o.precision_mask & (1u << f))) continue;
        const double u = UNIT[f];
        if ((u * u) * lhs <= rhs) {
            fmt = f;
            return;
        }
    }
    fmt = HH_FMT_FP64;
}

static void fill_stats(hh_handle* h, double seconds) {
    hh_stats& s = h->stats;
    s = hh_stats{};
    s.n = (int32_t)h->plan.n;
    s.d = h->plan.d;
    s.L = h->plan.L;
    s.ell = h->plan.ell;
    s.leaf_size = h->plan.leaf_size;
    double words = 0, words64 = 0, bytes = 0;
    for (const auto& r : h->blocks) {
        const int64_t m = r.b.ie - r.b.ib, n = r.b.je - r.b.jb;
        if (r.lowrank) {
            if (r.rank == 0) {
                s.n_blocks_rank0++;
                continue;
            }
            s.n_blocks_lowrank++;
            s.blocks_by_format[r.fmt]++;
            s.factor_bytes_by_format[r.fmt] +=
                (int64_t)r.rank * (col_bytes(r.fmt, r.t, r.PI) + col_bytes(r.fmt, r.t, r.PJ));
            s.lowrank_entries += (int64_t)r.rank * (m + n);
            s.total_columns += r.rank;
            s.max_rank = std::max(s.max_rank, r.rank);
            words += (double)r.rank * (m + n) * entry_bits(r.fmt, r.t) / 64.0;
            words64 += (double)r.rank * (m + n);
            bytes += (double)r.rank * (m + n) * entry_bits(r.fmt, r.t) / 8.0;
        } else {
            s.n_blocks_dense++;
            s.dense_entries += m * n;
            s.dense_bytes += r.PI * n * 8;
            words += (double)(m * n);
            words64 += (double)(m * n);
            bytes += 8.0 * m * n;
        }
    }
    const double io = h->opt.io_dtype == HH_IO_F32 ? 4.0 : 8.0;
    double vb = 0, ub = 0, db = 0;
    for (const auto& r : h->blocks) {
        const int64_t m = r.b.ie - r.b.ib, n = r.b.je - r.b.jb;
        if (r.lowrank) {
            vb += (double)r.rank * n * entry_bits(r.fmt, r.t) / 8.0;
            ub += (double)r.rank * m * entry_bits(r.fmt, r.t) / 8.0;
        } else {
            db += 8.0 * m * n;
        }
    }
    s.phase_bytes[0] = (io + 8.0) * h->plan.n;
    s.phase_bytes[1] = vb;
    s.phase_bytes[2] = ub + db + io * h->plan.n;
    s.storage_words = words;
    s.storage_words_fp64 = words64;
    s.matvec_bytes = bytes + 2.0 * io * h->plan.n;
    double t2 = 0;
    for (const auto& r : h->blocks)
        t2 += (r.lowrank && r.b.kind != HH_BLK_DENSE_NEAR) ? r.nb2 : r.entry2;
    s.norm2_total = t2;
    s.build_seconds = seconds;
}

// New task tables with the given sizes (0 = default); the tuner's step.
void retask(hh_handle* h, int64_t unit_bytes, int64_t dot_task_elems) {
    HIPCHK(hipDeviceSynchronize());
    h->unit_bytes = unit_bytes;
    h->dot_task_elems = dot_task_elems;
    build_tasks(h);
    ensure_part(h);
}

hh_handle* build_handle(const double* points, int64_t n, int d, const hh_kernel* k, double tol,
                        double eta, int switch_level, int leaf_size, const hh_options* opt) {
    auto t0 = std::chrono::steady_clock::now();
    if (!k) fail(HH_EINVAL, "kernel description is NULL");
    if (k->type < HH_LOG || k->type > HH_DOUBLE_LAYER) fail(HH_EINVAL, "unknown kernel type");
    if (!(tol > 0x1p-52 && tol < 1.0)) fail(HH_EINVAL, "tol must lie in (2^-52, 1)");
    if (k->type == HH_DOUBLE_LAYER && !k->normals) fail(HH_EINVAL, "double-layer kernel needs normals");
    if (!std::isfinite(k->scale) || !std::isfinite(k->h) || k->h < 0)
        fail(HH_EINVAL, "kernel scale and h must be finite, h >= 0");
    hh_options o{};
    o.precision_mask = 0xF;
    if (opt) o = *opt;
    if (o.precision_mask == 0) o.precision_mask = 0xF;
    if (o.precision_mask & ~0x2Fu) fail(HH_EINVAL, "precision_mask has bits outside 0x2F");
    if (o.io_dtype != HH_IO_F64 && o.io_dtype != HH_IO_F32) fail(HH_EINVAL, "io_dtype must be HH_IO_F64 or HH_IO_F32");
    if (o.continuum < 0 || o.continuum > 2) fail(HH_EINVAL, "continuum must be 0, 1 or 2");
    if (o.unit_bytes < 0 || o.dot_task_elems < 0) fail(HH_EINVAL, "task sizes must be >= 0");

    // wall time of each stage, printed when HH_VERBOSE is set
    auto tstage = t0;
    auto stage = [&](const char* what) {
        if (!Builder::verbose()) return;
        (void)hipDeviceSynchronize();
        const auto now = std::chrono::steady_clock::now();
        fprintf(stderr, "hh: build stage %-12s %8.3f s\n", what,
                std::chrono::duration<double>(now - tstage).count());
        fflush(stderr);
        tstage = now;
    };
    std::unique_ptr<hh_handle> h(new hh_handle());
    h->unit_bytes = o.unit_bytes;
    h->dot_task_elems = o.dot_task_elems;
    h->plan = make_plan(points, n, d, eta, switch_level, leaf_size);
    stage("plan");
    HIPCHK(hipGetDevice(&h->device));
    h->tol = tol;
    h->opt = o;
    h->kd = KernelDev{k->type, d, k->scale == 0.0 ? 1.0 : k->scale, k->h == 0.0 ? 1.0 : k->h};
    const Plan& P = h->plan;
    const bool uniform = o.uniform_fp64 != 0;

    // tree-ordered points (and normals) on the device
    std::vector<double> pt((size_t)n * d), nt;
    for (int64_t t = 0; t < n; ++t)
        for (int c = 0; c < d; ++c) pt[t * d + c] = points[P.perm[t] * d + c];
    h->d_pts = upload(h->mem, pt);
    if (k->type == HH_DOUBLE_LAYER) {
        nt.resize((size_t)n * d);
        for (int64_t t = 0; t < n; ++t)
            for (int c = 0; c < d; ++c) {
                double v = k->normals[P.perm[t] * d + c];
                if (!std::isfinite(v)) fail(HH_EINVAL, "normals must be finite");
                nt[t * d + c] = v;
            }
        h->d_nrm = upload(h->mem, nt);
    }
    layout(h.get());
    h->d_tpad = upload(h->mem, h->tpad);
    {
        std::vector<int64_t> pmap(h->np, -1);
        for (int64_t t = 0; t < n; ++t) pmap[h->tpad[t]] = P.perm[t];
        h->d_pmap = upload(h->mem, pmap);
    }

    stage("upload");
    Builder B(h.get());
    B.init();
    stage("init");
    std::vector<int64_t> cand, dense_list, near_adaptive;
    for (size_t i = 0; i < h->blocks.size(); ++i) {
        BlockRec& r = h->blocks[i];
        const int kind = r.b.kind;
        if (kind == HH_BLK_DIAG || (kind == HH_BLK_DENSE_NEAR && uniform)) {
            dense_list.push_back((int64_t)i);
        } else {
            r.lowrank = true;
            cand.push_back((int64_t)i);
            if (kind == HH_BLK_DENSE_NEAR) near_adaptive.push_back((int64_t)i);
        }
    }
    B.compress(cand);
    stage("compress");
    B.dense(dense_list);
    stage("dense");

    // Alg. 5: ||H~||^2; leaf neighbours of an H_s matrix enter with ||H_IJ||^2
    double total2 = 0.0;
    for (const auto& r : h->blocks) {
        if (r.b.kind == HH_BLK_DENSE_NEAR || !r.lowrank) total2 += r.entry2;
        else total2 += r.nb2;
    }
    // Alg. 3: storage precision per low-rank block
    std::vector<int64_t> to_dense;
    for (size_t i = 0; i < h->blocks.size(); ++i) {
        BlockRec& r = h->blocks[i];
        if (!r.lowrank) continue;
        int fmt = HH_FMT_FP64, t = 0;
        if (!uniform) choose_lowrank_format(r, total2, d, tol, o, fmt, t);
        r.fmt = fmt;
        r.t = t;
        if (r.b.kind == HH_BLK_DENSE_NEAR) {
            const int64_t m = r.b.ie - r.b.ib, nn = r.b.je - r.b.jb;
            // keep the neighbour low-rank only when that saves storage
            if (!((double)r.rank * (m + nn) * entry_bits(fmt, t) / 64.0 < (double)(m * nn)))
                to_dense.push_back((int64_t)i);
        }
    }
    for (int64_t i : to_dense) {
        BlockRec& r = h->blocks[i];
        double e2 = r.entry2;
        r.u_ptr = r.v_ptr = nullptr;
        B.dense({i});
        r.entry2 = e2;
        r.nb2 = e2;
    }
    B.pack();
    stage("pack");
    build_tasks(h.get());
    stage("tasks");
    h->ws_R = 1;
    h->xt = static_cast<double*>(h->mem.alloc((size_t)h->np * 8 + 256, true));
    h->tb = static_cast<double*>(h->mem.alloc((size_t)std::max<int64_t>(h->ncols, 1) * 8 + 256, true));
    ensure_part(h.get());
    if (h->all_fp64) {
        // the fp64 store chunks are the arena: hand their ownership to the handle
        for (void* p : B.store.ptrs) h->mem.ptrs.push_back(p);
        B.store.ptrs.clear();
    }
    HIPCHK(hipDeviceSynchronize());
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(h.get(), secs);
    return h.release();
}

}  // namespace hh

namespace hh {
// A handle with the source's tree, partition and fp64 factors re-stored under
// new options (Alg. 3 with another precision set, or uniform fp64).
hh_handle* derive_handle(const hh_handle* src, const hh_options* opt) {
    auto t0 = std::chrono::steady_clock::now();
    hh_options o{};
    o.precision_mask = 0xF;
    if (opt) o = *opt;
    if (o.precision_mask == 0) o.precision_mask = 0xF;
    if (o.precision_mask & ~0x2Fu) fail(HH_EINVAL, "precision_mask has bits outside 0x2F");
    if (o.io_dtype != HH_IO_F64 && o.io_dtype != HH_IO_F32) fail(HH_EINVAL, "io_dtype must be HH_IO_F64 or HH_IO_F32");
    if (o.continuum < 0 || o.continuum > 2) fail(HH_EINVAL, "continuum must be 0, 1 or 2");
    if (o.unit_bytes < 0 || o.dot_task_elems < 0) fail(HH_EINVAL, "task sizes must be >= 0");
    if (!src->all_fp64) fail(HH_ENOTSUP, "hh_derive needs a source whose factors are all fp64");
    for (const auto& r : src->blocks)
        if (r.b.kind == HH_BLK_DENSE_NEAR)
            fail(HH_ENOTSUP, "hh_derive does not support sources with ell == L");
    std::unique_ptr<hh_handle> h(new hh_handle());
    h->plan = src->plan;
    h->device = src->device;
    h->kd = src->kd;
    h->tol = src->tol;
    h->opt = o;
    h->np = src->np;
    h->leaf_poff = src->leaf_poff;
    h->leaf_psz = src->leaf_psz;
    h->tpad = src->tpad;
    h->blocks = src->blocks;
    h->unit_bytes = o.unit_bytes;
    h->dot_task_elems = o.dot_task_elems;
    for (auto& r : h->blocks) r.dt_ptr = nullptr;      // own transposed copies
    h->d_tpad = upload(h->mem, h->tpad);
    {
        std::vector<int64_t> pmap(h->np, -1);
        for (int64_t t = 0; t < h->plan.n; ++t) pmap[h->tpad[t]] = h->plan.perm[t];
        h->d_pmap = upload(h->mem, pmap);
    }
    // dense blocks: own copy
    int64_t total = 0;
    for (const auto& r : h->blocks)
        if (!r.lowrank) total += r.PI * (r.b.je - r.b.jb);
    double* D = static_cast<double*>(h->mem.alloc((size_t)total * 8 + 256, false));
    int64_t off = 0;
    for (auto& r : h->blocks) {
        if (r.lowrank) continue;
        const int64_t cnt = r.PI * (r.b.je - r.b.jb);
        HIPCHK(hipMemcpy(D + off, r.d_ptr, (size_t)cnt * 8, hipMemcpyDeviceToDevice));
        r.d_ptr = D + off;
        off += cnt;
    }
    const bool uniform = o.uniform_fp64 != 0;
    double total2 = 0.0;
    for (const auto& r : h->blocks) total2 += r.lowrank ? r.nb2 : r.entry2;
    for (auto& r : h->blocks) {
        if (!r.lowrank) continue;
        int fmt = HH_FMT_FP64, t = 0;
        if (!uniform) choose_lowrank_format(r, total2, h->plan.d, h->tol, o, fmt, t);
        r.fmt = fmt;
        r.t = t;
        r.eU = r.eV = 0;
    }
    Builder B(h.get());
    B.init((size_t)256 << 20);
    B.pack(false);              // reads the source's fp64 factors, writes own arenas
    build_tasks(h.get());
    h->ws_R = 1;
    h->xt = static_cast<double*>(h->mem.alloc((size_t)h->np * 8 + 256, true));
    h->tb = static_cast<double*>(h->mem.alloc((size_t)std::max<int64_t>(h->ncols, 1) * 8 + 256, true));
    ensure_part(h.get());
    HIPCHK(hipDeviceSynchronize());
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_stats(h.get(), secs);
    return h.release();
}
}  // namespace hh
