// Work items of the construction kernels (one item per block of a batch).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hh_internal.h"

namespace hh {

struct KernelDev {
    int type;
    int d;
    double scale;
    double h;
};

struct GenItem {
    int64_t ib, jb;      // tree-order start of rows / columns
    int64_t m, n;        // block size
    double* out;         // column-major destination
    int64_t ld;          // leading dimension of out
    int32_t mode;        // 0: compact rows, zero padding to M x N; 1: padded-row layout
    int32_t pad_;
};

struct SumItem {
    const double* ptr;
    int64_t count;
};

struct SketchItem {
    double* out;         // N x s column-major
    int64_t n;           // real rows
    int64_t uid;         // canonical block index
    int32_t round;       // sketch round (0 for width 32, +1 per doubling)
    int32_t pad_;
};

struct RankItem {
    const double* sigma; // p singular values, descending
    const double* norm2p;// ||H_b||_F^2 from the entries (device)
    const double* extrap;// ||H - Q B||_F^2 of the randomized path (device), or null
    int32_t p;           // number of singular values
    int32_t sketch;      // sketch width, 0 = exact SVD
    int32_t pmin;        // min(m, n) of the block
    int32_t oversample;
    // outputs
    int32_t rank;
    int32_t accept;
    double norm2, extra;
    double tail, tail_prev, trunc2;
};

struct FinItem {
    const double* U;     // m x >= k, column-major, leading dimension ldu
    const double* V;     // right factor: see v_rows
    const double* sigma;
    double* Uout;        // PI x k padded-row layout
    double* Vout;        // PJ x k padded-row layout
    int64_t ib, jb;
    int64_t ldu, ldv;
    int64_t PI, PJ;
    int32_t m, n, k;
    int32_t v_rows;      // 1: V holds V^T (singular index = row, ld ldv), times sigma;
                         // 0: V is n x k column-major (ld ldv), already scaled
};

// Householder QR (geqrf output) -> explicit Q (compact-WY helpers).
struct QrItem {
    const double* A;     // rows x s after geqrf (R above, reflectors below)
    const double* tau;   // s
    double* Vm;          // rows x s unit lower trapezoidal reflectors (0 column when tau = 0)
    double* R;           // s x s upper triangle of A, or null
    double* G;           // s x s, V^T V (input of the T kernel)
    double* Tinv;        // s x s: diag(1/tau) + strict upper part of G
    double* T;           // s x s: set to the identity (right-hand side of the solve)
    double* Q;           // rows x s: set to [I; 0]
    int64_t rows;
};

// One-sided Jacobi SVD of a small square matrix.
struct JacItem {
    double* A;           // s x s column-major: in A, out A J (columns sigma_r w_r), sorted
    double* J;           // s x s out: accumulated rotations (right singular vectors)
    double* sigma;       // s out, decreasing
};

// Transposed copy of a dense block: dst (rows n, ld_dst) = src^T for the
// m x n column-major src (ld_src); rows n .. ld_dst of dst stay zero.
struct TransItem {
    const double* src;
    double* dst;
    int64_t m, n;
    int64_t ld_src, ld_dst;
};

// Rows [0, rows_dst) of n columns into dst (ld_dst): src rows [0, m) (ld_src),
// zeros below.
struct CopyItem {
    const double* src;
    double* dst;
    int64_t m, n;
    int64_t ld_src, ld_dst;
    int64_t rows_dst;
};

struct PackItem {
    const double* src;
    void* dst;
    int64_t count;
    int32_t fmt;
    int32_t e;
};

// Continuum packing: k columns of P fp64 entries (padded-row layout) into k
// columns of cdw dwords, entries of 9 + t bits back to back.
struct ContPackItem {
    const double* src;
    uint32_t* dst;
    int64_t P;
    int64_t cdw;
    int32_t k;
    int32_t t;
};

__host__ __device__ uint16_t f64_to_f16_rne(double x);
__host__ __device__ uint16_t f64_to_bf16_rne(double x);
__host__ __device__ double f16_to_f64(uint16_t h);
__host__ __device__ double bf16_to_f64(uint16_t b);
__host__ __device__ uint8_t f64_to_q43_rne(double x);
__host__ __device__ double q43_to_f64(uint8_t c);
__host__ __device__ uint32_t f64_to_cont_rne(double x, int t);
__host__ __device__ double cont_to_f64(uint32_t code, int t);

void launch_gen(const KernelDev& k, const double* pts, const double* nrm, const int64_t* tpad,
                const GenItem* items, int nitems, int64_t M, int64_t N, int64_t max_total,
                hipStream_t s);
void launch_sumsq(const SumItem* items, int nitems, int64_t max_count, double* partial,
                  int64_t chunk, double* out, hipStream_t s);
void launch_sketch(const SketchItem* items, int nitems, int64_t N, int sk, uint64_t seed,
                   hipStream_t s);
void launch_rank(RankItem* items, int nitems, double eps2, hipStream_t s);
void launch_finalize(const FinItem* items, int nitems, const int64_t* tpad, hipStream_t s);
void launch_maxabs(const SumItem* items, int nitems, double* out, hipStream_t s);
void launch_pack(const PackItem* items, int nitems, int64_t max_count, hipStream_t s);
void launch_transpose(const TransItem* items, int nitems, int64_t max_count, hipStream_t s);
void launch_copy2d(const CopyItem* items, int nitems, int64_t max_count, hipStream_t s);
void launch_pack_cont(const ContPackItem* items, int nitems, int64_t max_dwords, hipStream_t s);
void launch_house_qr(double* A, int64_t ld, int64_t strideA, double* tau, int64_t strideT,
                     int64_t m, int n, int nitems, hipStream_t st);
void launch_panel_v(const double* A, int64_t ld, int64_t strideA, const double* tau,
                    int64_t strideT, double* V, double* T, int64_t m, int nb, int nitems,
                    hipStream_t st);
void launch_panel_tinv(const double* G, const double* tau, int64_t strideT, double* Tinv, int nb,
                       int nitems, hipStream_t st);
void launch_qr_extract(const QrItem* items, int nitems, int64_t rows, int s, hipStream_t st);
void launch_qr_tinv(const QrItem* items, int nitems, int s, hipStream_t st);
void launch_jacobi(const JacItem* items, int nitems, int s, hipStream_t st);
void launch_jacobi128(const JacItem* items, int nitems, int s, hipStream_t st);
// Tiled one-sided Jacobi for 128 < s <= 512; work: nitems x 2 s x jacobi_tiled_cols(s) doubles.
int jacobi_tiled_width(int s);
int jacobi_tiled_cols(int s);
void launch_jacobi_tiled(const JacItem* items, double* work, int nitems, int s, hipStream_t st);
void launch_svd_to_jac(const JacItem* items, const double* U, const double* Vt, int nitems, int s,
                       hipStream_t st);

}  // namespace hh
