// C ABI of the H_h library: argument checks, error reporting, products,
// inspection. Every entry point catches internal errors and returns a status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "handle.h"

namespace hh {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }
[[noreturn]] void fail(hh_status code, const std::string& msg) { throw Error{code, msg}; }

hh_handle* build_handle(const double* points, int64_t n, int d, const hh_kernel* k, double tol,
                        double eta, int switch_level, int leaf_size, const hh_options* opt);
hh_handle* derive_handle(const hh_handle* src, const hh_options* opt);

static size_t fmt_size(int fmt) {
    return fmt == HH_FMT_FP64 ? 8 : fmt == HH_FMT_FP32 ? 4 : fmt == HH_FMT_Q43 ? 1 : 2;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            fail(HH_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));                 \
    } while (0)

static void ensure_workspace(hh_handle* h, int64_t R) {
    if (R <= h->ws_R) return;
    void* xt = h->mem.alloc((size_t)h->np * R * 8 + 256, true);
    void* tb = h->mem.alloc((size_t)std::max<int64_t>(h->ncols, 1) * R * 8 + 256, true);
    h->mem.release(h->xt);
    h->mem.release(h->tb);
    h->xt = static_cast<double*>(xt);
    h->tb = static_cast<double*>(tb);
    h->ws_R = R;
}

static void check_device(const hh_handle* h) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != h->device) fail(HH_EINVAL, "the current device is not the handle's device");
}

static Desc make_desc(const hh_handle* h, const TaskSet& S, const void* x, void* y) {
    Desc d{};
    d.xt = h->xt;
    d.tb = h->tb;
    d.pmap = h->d_pmap;
    d.x = x;
    d.y = y;
    d.runs = S.d_runs;
    d.cl_run = S.d_cl_run;
    d.uruns = S.d_uruns;
    d.part = h->part;
    d.np = h->np;
    d.io = h->opt.io_dtype;
    d.d = h->plan.d;
    d.L = h->plan.L;
    return d;
}

static void product(const hh_handle* hc, const void* x, void* y, int64_t nrhs, void* stream,
                    bool trans, double* phase_ms = nullptr) {
    if (!hc) fail(HH_EINVAL, "handle is NULL");
    if (!x || !y) fail(HH_EINVAL, "x and y must be device pointers");
    if (x == y) fail(HH_EINVAL, "x and y must not alias");
    if (nrhs < 1 || nrhs > (1 << 16)) fail(HH_EINVAL, "nrhs must lie in [1, 65536]");
    check_device(hc);
    hh_handle* h = const_cast<hh_handle*>(hc);
    ensure_workspace(h, nrhs);
    const int R = (int)nrhs;
    const TaskSet& S = trans ? h->bwd : h->fwd;
    const Desc d = make_desc(h, S, x, y);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (phase_ms) {
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        HIPCHK(hipEventRecord(ev[0], (hipStream_t)stream));
    }
    launch_gather(d, nullptr, 1, h->np, R, stream);
    if (phase_ms) HIPCHK(hipEventRecord(ev[1], (hipStream_t)stream));
    if (R == 1 && S.dot_panel)
        launch_dot1_panel(d, nullptr, S.d_dot1p, (int64_t)S.dot1p.size(), h->family, stream);
    else if (R == 1) launch_dot(d, nullptr, S.d_dot, (int64_t)S.dot.size(), R, h->family, stream);
    else if (R <= PANEL_MAX_R && !h->has_cont)
        launch_dot(d, nullptr, S.d_dotp, (int64_t)S.dotp.size(), R, h->family, stream);
    else launch_dot(d, nullptr, S.d_dotm, (int64_t)S.dotm.size(), R, h->family, stream);
    if (phase_ms) HIPCHK(hipEventRecord(ev[2], (hipStream_t)stream));
    if (R == 1)
        launch_units(d, nullptr, S.d_unit, (int64_t)S.unit.size(), S.d_fin, (int64_t)S.fin.size(),
                     h->family, stream);
    else
        launch_accumulate(d, nullptr, S.d_leaf, (int64_t)S.leaf.size(), R, h->family, stream);
    HIPCHK(hipGetLastError());
    if (phase_ms) {
        HIPCHK(hipEventRecord(ev[3], (hipStream_t)stream));
        HIPCHK(hipEventSynchronize(ev[3]));
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            phase_ms[k] = ms;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
    }
}

// The product for the solver (same checks and kernels as hh_matvec).
void apply_product(const hh_handle* h, const void* x, void* y, int64_t nrhs, void* stream, bool trans) {
    product(h, x, y, nrhs, stream, trans);
}

void gmres(const hh_handle* h, const double* b, double* x, double shift, double rtol, int restart,
           int max_iter, int trans, int32_t* iters, double* relres, void* stream);

// Workspace of hh_matvec_noalloc: one fixed array per device. Host code never
// uses the array's name as an address: the device address is looked up once
// per device with hipGetSymbolAddress (that device current) and kept.
static __device__ __align__(256) unsigned char scratch[HH_NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES] = {};

static char* scratch_address(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) fail(HH_ENOTSUP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) fail(HH_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    return static_cast<char*>(g_scratch_ptr[dev]);
}

static int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

// The product of product() with the workspace carved from the device's scratch
// array: gathered x, coefficients, partial rows. Every element the kernels read
// is written earlier in the same call, so nothing is cleared.
static void product_noalloc(const hh_handle* h, const void* x, void* y, int64_t nrhs, bool trans,
                            void* stream) {
    if (!h) fail(HH_EINVAL, "handle is NULL");
    if (!x || !y) fail(HH_EINVAL, "x and y must be device pointers");
    if (x == y) fail(HH_EINVAL, "x and y must not alias");
    if (nrhs < 1 || nrhs > (1 << 16)) fail(HH_EINVAL, "nrhs must lie in [1, 65536]");
    check_device(h);
    const int R = (int)nrhs;
    const int64_t bx = round256(h->np * R * 8);
    const int64_t bt = round256(std::max<int64_t>(h->ncols, 1) * R * 8);
    const int64_t bp = R == 1 ? round256(std::max<int64_t>(h->part_rows, 1) * 8) : 0;
    if (bx + bt + bp > (int64_t)HH_NOALLOC_SCRATCH_BYTES)
        fail(HH_ENOTSUP, "the product needs " + std::to_string(bx + bt + bp) +
                             " bytes of workspace, more than the " +
                             std::to_string((long long)HH_NOALLOC_SCRATCH_BYTES) +
                             " of the allocation-free scratch");
    char* base = scratch_address(h->device);
    const TaskSet& S = trans ? h->bwd : h->fwd;
    Desc d = make_desc(h, S, x, y);
    d.xt = reinterpret_cast<double*>(base);
    d.tb = reinterpret_cast<double*>(base + bx);
    d.part = reinterpret_cast<double*>(base + bx + bt);
    launch_gather(d, nullptr, 1, h->np, R, stream);
    if (R == 1) {
        if (S.dot_panel)
            launch_dot1_panel(d, nullptr, S.d_dot1p, (int64_t)S.dot1p.size(), h->family, stream);
        else
            launch_dot(d, nullptr, S.d_dot, (int64_t)S.dot.size(), R, h->family, stream);
        launch_units(d, nullptr, S.d_unit, (int64_t)S.unit.size(), S.d_fin, (int64_t)S.fin.size(),
                     h->family, stream);
    } else {
        if (R <= PANEL_MAX_R && !h->has_cont)
            launch_dot(d, nullptr, S.d_dotp, (int64_t)S.dotp.size(), R, h->family, stream);
        else
            launch_dot(d, nullptr, S.d_dotm, (int64_t)S.dotm.size(), R, h->family, stream);
        launch_accumulate(d, nullptr, S.d_leaf, (int64_t)S.leaf.size(), R, h->family, stream);
    }
    HIPCHK(hipGetLastError());
}

// Task tables of the last batch (its handles and RHS count) stay on the
// device; a call with the same batch only uploads the descriptors (x, y and
// workspace pointers) on its stream. Freeing a member handle drops the plan.
struct BatchPlan {
    std::vector<const hh_handle*> hs;
    int64_t R = 0;
    int device = -1;
    DevMem mem;
    Desc* d_desc = nullptr;
    DotTask* d_dot = nullptr;
    LeafTask* d_leaf = nullptr;
    UnitTask* d_unit = nullptr;
    FinishTask* d_fin = nullptr;
    int64_t ndot = 0, nleaf = 0, nunit = 0, nfin = 0, max_np = 0;
};
static std::mutex g_batch_mu;
static std::unique_ptr<BatchPlan> g_batch;

template <class T>
static T* upload_to(DevMem& m, const std::vector<T>& v) {
    T* d = static_cast<T*>(m.alloc(v.size() * sizeof(T) + 16, false));
    if (!v.empty()) HIPCHK(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

static void product_batch(const hh_handle* const* hs, int count, const void* const* x,
                          void* const* y, int64_t nrhs, void* stream) {
    if (!hs || !x || !y || count < 1) fail(HH_EINVAL, "batch needs count >= 1 handles, x and y");
    if (nrhs < 1 || nrhs > (1 << 16)) fail(HH_EINVAL, "nrhs must lie in [1, 65536]");
    if (count > 65535) fail(HH_EINVAL, "at most 65535 handles per batch");
    const int io = hs[0] ? hs[0]->opt.io_dtype : 0;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    std::vector<Desc> descs(count);
    int fam = FAM_FIX;                       // q43 kernels also serve fixed-format handles
    for (int t = 0; t < count; ++t) {
        hh_handle* h = const_cast<hh_handle*>(hs[t]);
        if (!h) fail(HH_EINVAL, "a handle in the batch is NULL");
        if (!x[t] || !y[t] || x[t] == y[t]) fail(HH_EINVAL, "batch x / y pointers invalid");
        if (h->opt.io_dtype != io) fail(HH_EINVAL, "handles of a batch must share io_dtype");
        if (h->has_cont != hs[0]->has_cont)
            fail(HH_ENOTSUP, "a batch cannot mix continuum-stored and fixed-format handles");
        fam = std::max(fam, h->family);
        check_device(h);
        for (int u = 0; u < t; ++u)
            if (hs[u] == h) fail(HH_EINVAL, "a handle appears twice in the batch (shared workspace)");
        ensure_workspace(h, nrhs);
        descs[t] = make_desc(h, h->fwd, x[t], y[t]);
    }
    std::lock_guard<std::mutex> lock(g_batch_mu);
    BatchPlan* bp = g_batch.get();
    const bool same = bp && bp->R == nrhs && bp->device == dev && (int)bp->hs.size() == count &&
                      std::equal(bp->hs.begin(), bp->hs.end(), hs);
    if (!same) {
        g_batch.reset();
        std::unique_ptr<BatchPlan> np(new BatchPlan());
        np->hs.assign(hs, hs + count);
        np->R = nrhs;
        np->device = dev;
        std::vector<DotTask> dot;
        std::vector<LeafTask> leaf;
        std::vector<UnitTask> unit;
        std::vector<FinishTask> fin;
        for (int t = 0; t < count; ++t) {
            const hh_handle* h = hs[t];
            np->max_np = std::max(np->max_np, h->np);
            for (DotTask k : (nrhs == 1 ? h->fwd.dot
                              : nrhs <= PANEL_MAX_R && !hs[0]->has_cont ? h->fwd.dotp
                                                                         : h->fwd.dotm)) {
                k.hid = t;
                dot.push_back(k);
            }
            for (LeafTask k : h->fwd.leaf) {
                k.hid = t;
                leaf.push_back(k);
            }
            for (UnitTask k : h->fwd.unit) {
                k.hid = t;
                unit.push_back(k);
            }
            for (FinishTask k : h->fwd.fin) {
                k.hid = t;
                fin.push_back(k);
            }
        }
        np->d_desc = static_cast<Desc*>(np->mem.alloc(count * sizeof(Desc) + 16, false));
        np->d_dot = upload_to(np->mem, dot);
        np->d_leaf = upload_to(np->mem, leaf);
        np->d_unit = upload_to(np->mem, unit);
        np->d_fin = upload_to(np->mem, fin);
        np->ndot = (int64_t)dot.size();
        np->nleaf = (int64_t)leaf.size();
        np->nunit = (int64_t)unit.size();
        np->nfin = (int64_t)fin.size();
        g_batch = std::move(np);
        bp = g_batch.get();
    }
    HIPCHK(hipMemcpyAsync(bp->d_desc, descs.data(), count * sizeof(Desc), hipMemcpyHostToDevice,
                          (hipStream_t)stream));
    const int R = (int)nrhs;
    launch_gather(descs[0], bp->d_desc, count, bp->max_np, R, stream);
    launch_dot(descs[0], bp->d_desc, bp->d_dot, bp->ndot, R, fam, stream);
    if (R == 1)
        launch_units(descs[0], bp->d_desc, bp->d_unit, bp->nunit, bp->d_fin, bp->nfin, fam, stream);
    else
        launch_accumulate(descs[0], bp->d_desc, bp->d_leaf, bp->nleaf, R, fam, stream);
    HIPCHK(hipGetLastError());
}

static void drop_batch_plan(const hh_handle* h) {
    std::lock_guard<std::mutex> lock(g_batch_mu);
    if (g_batch && std::find(g_batch->hs.begin(), g_batch->hs.end(), h) != g_batch->hs.end())
        g_batch.reset();
}

// 64-bit words one stored block occupies: k (m + n) bits / 64 as factors,
// m n dense (the storage measure of eq:S1 / eq:S2, weighted by format bits).
static double block_words(const BlockRec& r) {
    const double m = (double)(r.b.ie - r.b.ib), n = (double)(r.b.je - r.b.jb);
    if (!r.lowrank) return m * n;
    const double bits = r.fmt == HH_FMT_FP64 ? 64.0 : r.fmt == HH_FMT_FP32 ? 32.0
                      : r.fmt == HH_FMT_CONT ? 9.0 + r.t : r.fmt == HH_FMT_Q43 ? 8.0 : 16.0;
    return (double)r.rank * (m + n) * bits / 64.0;
}

// Sec. 3.3, Alg. 2. H_s (switching level L) gives S1(ell) for every ell: its
// interaction lists of levels ell+1..L plus its leaf neighbours. Each H_h(ell)
// the walk reaches gives S2(ell): its compressed neighbours N_s(ell) plus its
// sibling lists of levels ell+1..L. The walk lowers ell from L while the gain
// S1 - S2 strictly grows.
static int switch_level_search(const double* points, int64_t n, int d, const hh_kernel* k,
                               double tol, double eta, int leaf_size, const hh_options* opt,
                               double* s1, double* s2, int cap) {
    const int L = make_plan(points, n, d, eta, -1, leaf_size).L;
    if ((s1 || s2) && cap < L + 1) fail(HH_EINVAL, "s1 / s2 need L + 1 entries");
    std::unique_ptr<hh_handle, void (*)(hh_handle*)> hs(
        build_handle(points, n, d, k, tol, eta, L, leaf_size, opt), hh_free);
    std::vector<double> far(L + 2, 0.0), S1(L + 1), S2(L + 1, std::nan(""));
    double near_leaf = 0.0;
    for (const auto& r : hs->blocks) {
        if (r.b.kind == HH_BLK_FAR) far[r.b.level] += block_words(r);
        else if (r.b.kind == HH_BLK_DENSE_NEAR) near_leaf += block_words(r);
    }
    hs.reset();
    for (int ell = L; ell >= 0; --ell) S1[ell] = (ell == L ? 0.0 : S1[ell + 1] + far[ell + 1]);
    for (int ell = 0; ell <= L; ++ell) S1[ell] += near_leaf;
    S2[L] = S1[L];
    int ell = L;
    double gain = 0.0;
    while (ell > 0) {
        std::unique_ptr<hh_handle, void (*)(hh_handle*)> hb(
            build_handle(points, n, d, k, tol, eta, ell - 1, leaf_size, opt), hh_free);
        double w = 0.0;
        for (const auto& r : hb->blocks)
            if (r.b.kind == HH_BLK_NEAR || r.b.kind == HH_BLK_WEAK) w += block_words(r);
        S2[ell - 1] = w;
        const double g = S1[ell - 1] - w;
        if (g <= gain) break;
        gain = g;
        --ell;
    }
    if (s1) std::copy(S1.begin(), S1.end(), s1);
    if (s2) std::copy(S2.begin(), S2.end(), s2);
    return ell;
}

// Entry i of a continuum column of (9 + t)-bit entries packed back to back
// (little-endian bit order) from the column's first byte.
static double decode_cont(const unsigned char* col, int t, int64_t i) {
    const int w = 9 + t;
    const int64_t bit = i * w;
    uint64_t win = 0;
    for (int b = 0; b < 8; ++b) win |= (uint64_t)col[(bit >> 3) + b] << (8 * b);
    const uint32_t code = (uint32_t)((win >> (bit & 7)) & ((1ull << w) - 1));
    return cont_to_f64(code, t);
}

void retask(hh_handle* h, int64_t unit_bytes, int64_t dot_task_elems);

// Median milliseconds of one product (HIP events on the stream), after a
// warm-up product.
static double time_product(hh_handle* h, const void* x, void* y, void* stream) {
    product(h, x, y, 1, stream, false);
    std::vector<double> ms;
    for (int r = 0; r < 5; ++r) {
        double ph[3];
        product(h, x, y, 1, stream, false, ph);
        ms.push_back(ph[0] + ph[1] + ph[2]);
    }
    std::sort(ms.begin(), ms.end());
    return ms[2];
}

// Coordinate search over the single-vector task sizes (unit size, then
// inner-product task size); the handle keeps the fastest tables.
static void autotune(hh_handle* h, void* stream, hh_tuning* best, hh_tuning* tried, int32_t cap,
                     int32_t* ntried) {
    drop_batch_plan(h);
    const size_t io = h->opt.io_dtype == HH_IO_F32 ? 4 : 8;
    DevMem tmp;
    void* x = tmp.alloc((size_t)h->plan.n * io + 256, true);
    void* y = tmp.alloc((size_t)h->plan.n * io + 256, true);
    ensure_workspace(h, 1);
    std::vector<hh_tuning> log;
    auto trial = [&](int64_t ub, int64_t de) {
        retask(h, ub, de);
        hh_tuning t{ub, de, time_product(h, x, y, stream)};
        log.push_back(t);
        return t;
    };
    hh_tuning b{0, 0, 1e300};
    for (int64_t ub : {256LL << 10, 512LL << 10, 1LL << 20, 2LL << 20, 4LL << 20}) {
        const hh_tuning t = trial(ub, 65536);
        if (t.ms < b.ms) b = t;
    }
    for (int64_t de : {16384LL, 32768LL, 131072LL, 262144LL}) {
        const hh_tuning t = trial(b.unit_bytes, de);
        if (t.ms < b.ms) b = t;
    }
    retask(h, b.unit_bytes, b.dot_task_elems);
    HIPCHK(hipDeviceSynchronize());
    *best = b;
    if (tried)
        for (size_t i = 0; i < log.size() && (int32_t)i < cap; ++i) tried[i] = log[i];
    if (ntried) *ntried = (int32_t)log.size();
}

static double decode(const void* base, int fmt, int64_t i) {
    switch (fmt) {
        case HH_FMT_FP64: return static_cast<const double*>(base)[i];
        case HH_FMT_FP32: return static_cast<const float*>(base)[i];
        case HH_FMT_FP16: return f16_to_f64(static_cast<const uint16_t*>(base)[i]);
        case HH_FMT_Q43: return q43_to_f64(static_cast<const uint8_t*>(base)[i]);
        default: return bf16_to_f64(static_cast<const uint16_t*>(base)[i]);
    }
}

}  // namespace hh

using namespace hh;

#define GUARD_BEGIN try {
#define GUARD_END                                                                          \
    }                                                                                      \
    catch (const hh::Error& e) {                                                           \
        hh::set_error(e.msg);                                                              \
        return e.code;                                                                     \
    }                                                                                      \
    catch (const std::bad_alloc&) {                                                        \
        hh::set_error("host allocation failed");                                          \
        return HH_ENOMEM;                                                                  \
    }                                                                                      \
    catch (const std::exception& e) {                                                      \
        hh::set_error(e.what());                                                           \
        return HH_EINTERNAL;                                                               \
    }                                                                                      \
    hh::set_error("");                                                                     \
    return HH_OK;

extern "C" {

hh_status hh_build(const double* points, int64_t n, int d, const hh_kernel* k, double tol,
                   double eta, int switch_level, int leaf_size, const hh_options* opt,
                   hh_handle** out) {
    if (out) *out = nullptr;
    GUARD_BEGIN
    if (!out) fail(HH_EINVAL, "out is NULL");
    if (!points) fail(HH_EINVAL, "points is NULL");
    *out = build_handle(points, n, d, k, tol, eta, switch_level, leaf_size, opt);
    GUARD_END
}

hh_status hh_derive(const hh_handle* src, const hh_options* opt, hh_handle** out) {
    if (out) *out = nullptr;
    GUARD_BEGIN
    if (!out || !src) fail(HH_EINVAL, "src and out must not be NULL");
    check_device(src);
    *out = derive_handle(src, opt);
    GUARD_END
}

hh_status hh_switch_level_search(const double* points, int64_t n, int d, const hh_kernel* k,
                                 double tol, double eta, int leaf_size, const hh_options* opt,
                                 int32_t* level_out, double* s1, double* s2, int32_t cap) {
    GUARD_BEGIN
    if (!level_out) fail(HH_EINVAL, "level_out is NULL");
    if (!points) fail(HH_EINVAL, "points is NULL");
    *level_out = -1;
    *level_out = switch_level_search(points, n, d, k, tol, eta, leaf_size, opt, s1, s2, cap);
    GUARD_END
}

hh_status hh_matvec(const hh_handle* h, const void* x, void* y, int64_t nrhs, void* stream) {
    GUARD_BEGIN
    product(h, x, y, nrhs, stream, false);
    GUARD_END
}

hh_status hh_matvec_t(const hh_handle* h, const void* x, void* y, int64_t nrhs, void* stream) {
    GUARD_BEGIN
    product(h, x, y, nrhs, stream, true);
    GUARD_END
}

hh_status hh_matvec_timed(const hh_handle* h, const void* x, void* y, int64_t nrhs, void* stream,
                          int trans, double* phase_ms) {
    GUARD_BEGIN
    if (!phase_ms) fail(HH_EINVAL, "phase_ms is NULL");
    product(h, x, y, nrhs, stream, trans != 0, phase_ms);
    GUARD_END
}

hh_status hh_matvec_batch(const hh_handle* const* hs, int count, const void* const* x,
                          void* const* y, int64_t nrhs, void* stream) {
    GUARD_BEGIN
    product_batch(hs, count, x, y, nrhs, stream);
    GUARD_END
}

hh_status hh_matvec_noalloc(const hh_handle* h, const void* x, void* y, int64_t nrhs, int trans,
                            void* stream) {
    GUARD_BEGIN
    product_noalloc(h, x, y, nrhs, trans != 0, stream);
    GUARD_END
}

hh_status hh_solve(const hh_handle* h, const void* b, void* x, double shift, double rtol,
                   int restart, int max_iter, int trans, int32_t* iters, double* relres,
                   void* stream) {
    GUARD_BEGIN
    if (h) check_device(h);
    gmres(h, static_cast<const double*>(b), static_cast<double*>(x), shift, rtol, restart, max_iter,
          trans, iters, relres, stream);
    GUARD_END
}

hh_status hh_autotune(hh_handle* h, void* stream, hh_tuning* best, hh_tuning* tried, int32_t cap,
                      int32_t* ntried) {
    GUARD_BEGIN
    if (!h || !best) fail(HH_EINVAL, "handle and best must not be NULL");
    if (tried && cap < 0) fail(HH_EINVAL, "cap must be >= 0");
    check_device(h);
    autotune(h, stream, best, tried, cap, ntried);
    GUARD_END
}

hh_status hh_reserve(hh_handle* h, int64_t max_nrhs) {
    GUARD_BEGIN
    if (!h) fail(HH_EINVAL, "handle is NULL");
    if (max_nrhs < 1 || max_nrhs > (1 << 16)) fail(HH_EINVAL, "max_nrhs must lie in [1, 65536]");
    check_device(h);
    ensure_workspace(h, max_nrhs);
    GUARD_END
}

hh_status hh_get_stats(const hh_handle* h, hh_stats* out) {
    GUARD_BEGIN
    if (!h || !out) fail(HH_EINVAL, "NULL argument");
    *out = h->stats;
    GUARD_END
}

hh_status hh_block_count(const hh_handle* h, int64_t* count) {
    GUARD_BEGIN
    if (!h || !count) fail(HH_EINVAL, "NULL argument");
    *count = (int64_t)h->blocks.size();
    GUARD_END
}

hh_status hh_get_block(const hh_handle* h, int64_t index, hh_block_info* o) {
    GUARD_BEGIN
    if (!h || !o) fail(HH_EINVAL, "NULL argument");
    if (index < 0 || index >= (int64_t)h->blocks.size()) fail(HH_EINVAL, "block index out of range");
    const BlockRec& r = h->blocks[index];
    *o = hh_block_info{};
    o->level = r.b.level;
    o->kind = r.lowrank ? r.b.kind : (r.b.kind == HH_BLK_DIAG ? HH_BLK_DIAG : HH_BLK_DENSE_NEAR);
    o->rank = r.lowrank ? r.rank : 0;
    o->format = r.fmt;
    o->box_i = r.b.bi;
    o->box_j = r.b.bj;
    o->row_begin = r.b.ib;
    o->row_end = r.b.ie;
    o->col_begin = r.b.jb;
    o->col_end = r.b.je;
    o->exp_u = r.eU;
    o->exp_v = r.eV;
    o->lowrank = r.lowrank ? 1 : 0;
    o->frac_bits = r.lowrank && r.fmt == HH_FMT_CONT ? r.t : 0;
    o->norm2 = r.nb2;
    o->entry_norm2 = r.entry2;
    o->tail_prev = r.tail_prev;
    o->tail = r.tail;
    GUARD_END
}

hh_status hh_get_block_factors(const hh_handle* h, int64_t index, double* U, double* V) {
    GUARD_BEGIN
    if (!h || !U) fail(HH_EINVAL, "NULL argument");
    if (index < 0 || index >= (int64_t)h->blocks.size()) fail(HH_EINVAL, "block index out of range");
    check_device(h);
    HIPCHK(hipDeviceSynchronize());
    const BlockRec& r = h->blocks[index];
    const int64_t m = r.b.ie - r.b.ib, n = r.b.je - r.b.jb;
    const int64_t rb = h->tpad[r.b.ib], cb = h->tpad[r.b.jb];
    if (!r.lowrank) {
        std::vector<double> D((size_t)r.PI * n);
        HIPCHK(hipMemcpy(D.data(), r.d_ptr, D.size() * 8, hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) U[i + j * m] = D[j * r.PI + h->tpad[r.b.ib + i] - rb];
    } else if (r.rank > 0 && r.fmt == HH_FMT_CONT) {
        if (!V) fail(HH_EINVAL, "V is NULL for a low-rank block");
        const int64_t cu = cont_col_bytes(r.PI, 9 + r.t), cv = cont_col_bytes(r.PJ, 9 + r.t);
        std::vector<unsigned char> bu((size_t)r.rank * cu + 16, 0), bv((size_t)r.rank * cv + 16, 0);
        HIPCHK(hipMemcpy(bu.data(), r.u_ptr, (size_t)r.rank * cu, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(bv.data(), r.v_ptr, (size_t)r.rank * cv, hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < r.rank; ++c) {
            for (int64_t i = 0; i < m; ++i)
                U[i + c * m] = decode_cont(bu.data() + c * cu, r.t, h->tpad[r.b.ib + i] - rb);
            for (int64_t j = 0; j < n; ++j)
                V[j + c * n] = decode_cont(bv.data() + c * cv, r.t, h->tpad[r.b.jb + j] - cb);
        }
    } else if (r.rank > 0) {
        if (!V) fail(HH_EINVAL, "V is NULL for a low-rank block");
        const size_t es = fmt_size(r.fmt);
        std::vector<char> bu((size_t)r.rank * r.PI * es), bv((size_t)r.rank * r.PJ * es);
        HIPCHK(hipMemcpy(bu.data(), r.u_ptr, bu.size(), hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(bv.data(), r.v_ptr, bv.size(), hipMemcpyDeviceToHost));
        const double su = std::ldexp(1.0, r.eU), sv = std::ldexp(1.0, r.eV);
        for (int64_t c = 0; c < r.rank; ++c) {
            for (int64_t i = 0; i < m; ++i)
                U[i + c * m] = su * decode(bu.data(), r.fmt, c * r.PI + h->tpad[r.b.ib + i] - rb);
            for (int64_t j = 0; j < n; ++j)
                V[j + c * n] = sv * decode(bv.data(), r.fmt, c * r.PJ + h->tpad[r.b.jb + j] - cb);
        }
    }
    GUARD_END
}

hh_status hh_get_perm(const hh_handle* h, int64_t* perm) {
    GUARD_BEGIN
    if (!h || !perm) fail(HH_EINVAL, "NULL argument");
    std::memcpy(perm, h->plan.perm.data(), h->plan.perm.size() * sizeof(int64_t));
    GUARD_END
}

int hh_io_dtype(const hh_handle* h) { return h ? h->opt.io_dtype : -1; }
int64_t hh_size(const hh_handle* h) { return h ? h->plan.n : -1; }

void hh_free(hh_handle* h) {
    if (!h) return;
    int prev = -1;
    const int dev = h->device;
    (void)hipGetDevice(&prev);
    if (prev != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    drop_batch_plan(h);
    delete h;
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
}

hh_status hh_plan_create(const double* points, int64_t n, int d, double eta, int switch_level,
                         int leaf_size, hh_plan** out) {
    if (out) *out = nullptr;
    GUARD_BEGIN
    if (!out || !points) fail(HH_EINVAL, "NULL argument");
    hh_plan* p = new hh_plan();
    try {
        p->p = make_plan(points, n, d, eta, switch_level, leaf_size);
    } catch (...) {
        delete p;
        throw;
    }
    *out = p;
    GUARD_END
}

hh_status hh_plan_info(const hh_plan* p, int32_t* L, int32_t* ell, int64_t* n_blocks) {
    GUARD_BEGIN
    if (!p) fail(HH_EINVAL, "plan is NULL");
    if (L) *L = p->p.L;
    if (ell) *ell = p->p.ell;
    if (n_blocks) *n_blocks = (int64_t)p->p.blocks.size();
    GUARD_END
}

hh_status hh_plan_blocks(const hh_plan* p, int32_t* level, int32_t* kind, int64_t* box_i,
                         int64_t* box_j, int64_t* ib, int64_t* ie, int64_t* jb, int64_t* je) {
    GUARD_BEGIN
    if (!p) fail(HH_EINVAL, "plan is NULL");
    const auto& B = p->p.blocks;
    for (size_t i = 0; i < B.size(); ++i) {
        if (level) level[i] = B[i].level;
        if (kind) kind[i] = B[i].kind;
        if (box_i) box_i[i] = B[i].bi;
        if (box_j) box_j[i] = B[i].bj;
        if (ib) ib[i] = B[i].ib;
        if (ie) ie[i] = B[i].ie;
        if (jb) jb[i] = B[i].jb;
        if (je) je[i] = B[i].je;
    }
    GUARD_END
}

hh_status hh_plan_perm(const hh_plan* p, int64_t* perm) {
    GUARD_BEGIN
    if (!p || !perm) fail(HH_EINVAL, "NULL argument");
    std::memcpy(perm, p->p.perm.data(), p->p.perm.size() * sizeof(int64_t));
    GUARD_END
}

void hh_plan_free(hh_plan* p) { delete p; }

hh_status hh_quantize(const double* in, int64_t n, int format, int e, double* out) {
    GUARD_BEGIN
    if (n < 0 || (n > 0 && (!in || !out))) fail(HH_EINVAL, "bad arrays");
    if (format < HH_FMT_FP64 || format > HH_FMT_Q43 || format == HH_FMT_CONT)
        fail(HH_EINVAL, "unknown format");
    const double s = std::ldexp(1.0, -e), b = std::ldexp(1.0, e);
    for (int64_t i = 0; i < n; ++i) {
        double v = in[i] * s, q;
        switch (format) {
            case HH_FMT_FP64: q = v; break;
            case HH_FMT_FP32: q = (double)(float)v; break;
            case HH_FMT_FP16: q = f16_to_f64(f64_to_f16_rne(v)); break;
            case HH_FMT_Q43: q = q43_to_f64(f64_to_q43_rne(v)); break;
            default: q = bf16_to_f64(f64_to_bf16_rne(v)); break;
        }
        out[i] = q * b;
    }
    GUARD_END
}

hh_status hh_quantize_cont(const double* in, int64_t n, int t, double* out) {
    GUARD_BEGIN
    if (n < 0 || (n > 0 && (!in || !out))) fail(HH_EINVAL, "bad arrays");
    if (t < 7 || t > 23) fail(HH_EINVAL, "fraction bits must lie in [7, 23]");
    for (int64_t i = 0; i < n; ++i) out[i] = cont_to_f64(f64_to_cont_rne(in[i], t), t);
    GUARD_END
}

const char* hh_last_error(void) { return g_error.c_str(); }

}  // extern "C"
