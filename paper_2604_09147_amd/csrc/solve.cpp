// Iterative solution with the H_h product (the closing remark of Sec. 5.3: the
// fast mixed-precision product serves iterative solvers): restarted GMRES
// (Saad & Schultz, 1986) for (H^ + shift I) x = b on the device. The operator
// is the library's own product; the Krylov basis is made orthonormal by
// classical Gram-Schmidt applied twice (two pairs of rocBLAS GEMVs per
// step); the small Hessenberg least-squares problem is kept triangular with
// Givens rotations on the host.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cmath>
#include <string>
#include <vector>

#include "handle.h"

namespace hh {

void apply_product(const hh_handle* h, const void* x, void* y, int64_t nrhs, void* stream, bool trans);

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
            fail(HH_EHIP, std::string(#x) + ": rocblas status " + std::to_string((int)s_)); \
    } while (0)

namespace {
struct Blas {
    rocblas_handle rb = nullptr;
    ~Blas() {
        if (rb) rocblas_destroy_handle(rb);
    }
};
}  // namespace

void gmres(const hh_handle* h, const double* b, double* x, double shift, double rtol, int restart,
           int max_iter, int trans, int32_t* iters, double* relres, void* stream) {
    if (!h || !b || !x) fail(HH_EINVAL, "handle, b and x must not be NULL");
    if (b == x) fail(HH_EINVAL, "b and x must not alias");
    if (h->opt.io_dtype != HH_IO_F64) fail(HH_ENOTSUP, "the solver works on handles with fp64 io");
    if (!(rtol > 0.0) || !std::isfinite(shift)) fail(HH_EINVAL, "rtol must be > 0 and shift finite");
    if (restart < 1 || restart > 1000) fail(HH_EINVAL, "restart must lie in [1, 1000]");
    if (max_iter < 0) fail(HH_EINVAL, "max_iter must be >= 0");
    const int64_t n = h->plan.n;
    const int m = restart;
    const hipStream_t st = (hipStream_t)stream;
    DevMem mem;
    double* V = static_cast<double*>(mem.alloc((size_t)n * (m + 1) * 8, false));
    double* w = static_cast<double*>(mem.alloc((size_t)n * 8, false));
    double* hv = static_cast<double*>(mem.alloc((size_t)(m + 2) * 2 * 8, false));
    Blas B;
    RBCHK(rocblas_create_handle(&B.rb));
    RBCHK(rocblas_set_stream(B.rb, st));
    RBCHK(rocblas_set_pointer_mode(B.rb, rocblas_pointer_mode_host));
    RBCHK(rocblas_set_atomics_mode(B.rb, rocblas_atomics_not_allowed));
    const double one = 1.0, mone = -1.0, zero = 0.0;
    // out = (H^ + shift I) v (or its transpose)
    auto apply = [&](const double* v, double* out) {
        apply_product(h, v, out, 1, stream, trans != 0);
        if (shift != 0.0) RBCHK(rocblas_daxpy(B.rb, (rocblas_int)n, &shift, v, 1, out, 1));
    };
    auto nrm2 = [&](const double* v) {
        double r = 0.0;
        RBCHK(rocblas_dnrm2(B.rb, (rocblas_int)n, v, 1, &r));
        return r;
    };
    const double nb = nrm2(b);
    if (iters) *iters = 0;
    if (nb == 0.0) {
        HIPCHK(hipMemsetAsync(x, 0, (size_t)n * 8, st));
        HIPCHK(hipStreamSynchronize(st));
        if (relres) *relres = 0.0;
        return;
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hh(m + 1), h2(m + 1), y(m);
    int it = 0;
    double res = 0.0;
    while (true) {
        // r = b - A x in V[:, 0]
        apply(x, w);
        HIPCHK(hipMemcpyAsync(V, b, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
        RBCHK(rocblas_daxpy(B.rb, (rocblas_int)n, &mone, w, 1, V, 1));
        const double beta = nrm2(V);
        res = beta / nb;
        if (res <= rtol || it >= max_iter) break;
        const double ib = 1.0 / beta;
        RBCHK(rocblas_dscal(B.rb, (rocblas_int)n, &ib, V, 1));
        const int mm = std::min(m, max_iter - it);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < mm; ++j) {
            double* vj = V + (int64_t)j * n;
            apply(vj, w);
            const rocblas_int cols = j + 1;
            // two passes of classical Gram-Schmidt: h = V^T w, w -= V h
            RBCHK(rocblas_dgemv(B.rb, rocblas_operation_transpose, (rocblas_int)n, cols, &one, V,
                                (rocblas_int)n, w, 1, &zero, hv, 1));
            RBCHK(rocblas_dgemv(B.rb, rocblas_operation_none, (rocblas_int)n, cols, &mone, V,
                                (rocblas_int)n, hv, 1, &one, w, 1));
            RBCHK(rocblas_dgemv(B.rb, rocblas_operation_transpose, (rocblas_int)n, cols, &one, V,
                                (rocblas_int)n, w, 1, &zero, hv + (m + 2), 1));
            RBCHK(rocblas_dgemv(B.rb, rocblas_operation_none, (rocblas_int)n, cols, &mone, V,
                                (rocblas_int)n, hv + (m + 2), 1, &one, w, 1));
            HIPCHK(hipMemcpyAsync(hh.data(), hv, cols * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(h2.data(), hv + (m + 2), cols * 8, hipMemcpyDeviceToHost, st));
            const double hn = nrm2(w);
            HIPCHK(hipStreamSynchronize(st));           // hh, h2 have arrived
            double* Hj = H.data() + (size_t)j * (m + 1);
            for (int i = 0; i <= j; ++i) Hj[i] = hh[i] + h2[i];
            Hj[j + 1] = hn;
            if (hn > 0.0) {
                const double ih = 1.0 / hn;
                HIPCHK(hipMemcpyAsync(vj + n, w, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
                RBCHK(rocblas_dscal(B.rb, (rocblas_int)n, &ih, vj + n, 1));
            }
            for (int i = 0; i < j; ++i) {
                const double a = Hj[i], c = Hj[i + 1];
                Hj[i] = cs[i] * a + sn[i] * c;
                Hj[i + 1] = -sn[i] * a + cs[i] * c;
            }
            const double a = Hj[j], c = Hj[j + 1];
            const double d = std::hypot(a, c);
            cs[j] = d == 0.0 ? 1.0 : a / d;
            sn[j] = d == 0.0 ? 0.0 : c / d;
            Hj[j] = d;
            Hj[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            k = j + 1;
            if (std::fabs(g[j + 1]) / nb <= rtol || hn == 0.0) break;
        }
        // y = R^-1 g, x += V[:, :k] y
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[(size_t)l * (m + 1) + i] * y[l];
            y[i] = s / H[(size_t)i * (m + 1) + i];
        }
        HIPCHK(hipMemcpyAsync(hv, y.data(), k * 8, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        RBCHK(rocblas_dgemv(B.rb, rocblas_operation_none, (rocblas_int)n, k, &one, V, (rocblas_int)n,
                            hv, 1, &one, x, 1));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (iters) *iters = it;
    if (relres) *relres = res;
}

}  // namespace hh
