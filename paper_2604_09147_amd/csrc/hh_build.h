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
    const double* Vt;    // >= k x n, column-major, leading dimension ldv (rows = singular index)
    const double* sigma;
    double* Uout;        // PI x k padded-row layout
    double* Vout;        // PJ x k padded-row layout
    int64_t ib, jb;
    int64_t ldu, ldv;
    int64_t PI, PJ;
    int32_t m, n, k, pad_;
};

struct PackItem {
    const double* src;
    void* dst;
    int64_t count;
    int32_t fmt;
    int32_t e;
};

__host__ __device__ uint16_t f64_to_f16_rne(double x);
__host__ __device__ uint16_t f64_to_bf16_rne(double x);
__host__ __device__ double f16_to_f64(uint16_t h);
__host__ __device__ double bf16_to_f64(uint16_t b);

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

}  // namespace hh
