// Device kernels of the construction stage (Alg. 1, Alg. 5, Alg. 3):
// kernel-matrix entries, Frobenius sums, Rademacher sketches, rank choice,
// factor finalisation and rounding into the storage formats.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hh_build.h"

namespace hh {

// --------------------------------------------------------------- rounding
// Round-to-nearest-even from float64 straight to the storage format (no
// detour through fp32, which would round twice).
__host__ __device__ uint16_t f64_to_f16_rne(double x) {
    const uint64_t bits = __builtin_bit_cast(uint64_t, x);
    uint16_t sign = (uint16_t)((bits >> 48) & 0x8000u);
    int ex = (int)((bits >> 52) & 0x7FF);
    uint64_t man = bits & ((1ull << 52) - 1);
    if (ex == 0x7FF) return sign | 0x7C00u | (man ? 0x200u : 0u);
    if (ex == 0) return sign;                       // |x| < 2^-1022 rounds to 0
    int e = ex - 1023;                              // x = M 2^(e - 52), M in [2^52, 2^53)
    if (e > 15) return sign | 0x7C00u;
    uint64_t M = man | (1ull << 52);
    int ue = (e > -14 ? e : -14) - 10;              // exponent of the fp16 ulp at |x|
    int shift = 52 + ue - e;                        // >= 42
    if (shift >= 64) return sign;
    uint64_t q = M >> shift;
    uint64_t rem = M & ((1ull << shift) - 1);
    uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    uint32_t out = e >= -14 ? (uint32_t)((e + 15) << 10) + (uint32_t)q - 1024u : (uint32_t)q;
    if (out >= 0x7C00u) out = 0x7C00u;
    return sign | (uint16_t)out;
}

__host__ __device__ uint16_t f64_to_bf16_rne(double x) {
    const uint64_t bits = __builtin_bit_cast(uint64_t, x);
    uint16_t sign = (uint16_t)((bits >> 48) & 0x8000u);
    int ex = (int)((bits >> 52) & 0x7FF);
    uint64_t man = bits & ((1ull << 52) - 1);
    if (ex == 0x7FF) return sign | 0x7F80u | (man ? 0x40u : 0u);
    if (ex == 0) return sign;
    int e = ex - 1023;
    if (e > 127) return sign | 0x7F80u;
    uint64_t M = man | (1ull << 52);
    int ue = (e > -126 ? e : -126) - 7;
    int shift = 52 + ue - e;                        // >= 45
    if (shift >= 64) return sign;
    uint64_t q = M >> shift;
    uint64_t rem = M & ((1ull << shift) - 1);
    uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    uint32_t out = e >= -126 ? (uint32_t)((e + 127) << 7) + (uint32_t)q - 128u : (uint32_t)q;
    if (out >= 0x7F80u) out = 0x7F80u;
    return sign | (uint16_t)out;
}

__host__ __device__ double f16_to_f64(uint16_t h) {
    int ex = (h >> 10) & 0x1F, man = h & 0x3FF;
    double v;
    if (ex == 0) v = ldexp((double)man, -24);
    else if (ex == 31) v = man ? NAN : INFINITY;
    else v = ldexp((double)(man | 0x400), ex - 25);
    return (h & 0x8000) ? -v : v;
}

__host__ __device__ double bf16_to_f64(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    return (double)__builtin_bit_cast(float, u);
}

// ------------------------------------------------------- kernel entries
// eq:kernel_mat: H_ij = scale f(|p_i - p_j|); singular kernels give 0 on the
// diagonal and for coincident points.
__device__ inline double kernel_entry(const KernelDev& k, const double* pts,
                                      const double* nrm, int64_t gi, int64_t gj) {
    const int d = k.d;
    double r2 = 0.0, dn = 0.0;
    for (int c = 0; c < d; ++c) {
        double df = pts[gi * d + c] - pts[gj * d + c];
        r2 += df * df;
        if (k.type == HH_DOUBLE_LAYER) dn += nrm[gj * d + c] * df;
    }
    double r = sqrt(r2);
    bool sing = k.type != HH_GAUSS && k.type != HH_MATERN;
    if (sing && (gi == gj || r == 0.0)) return 0.0;
    double v;
    switch (k.type) {
        case HH_LOG: v = log(r); break;
        case HH_INV_R: v = 1.0 / r; break;
        case HH_INV_R2: v = 1.0 / r2; break;
        case HH_GAUSS: v = exp(-r2 / (k.h * k.h)); break;
        case HH_MATERN: v = exp(-r / k.h); break;
        default: v = dn / (r2 * r); break;
    }
    return k.scale * v;
}

// One work item per block: out is column-major with leading dimension ld.
// mode 0: rows i < m at row i, entries outside m x n set to 0 (rows < M, cols < N).
// mode 1: row i at padded slot tpad[ib + i] - tpad[ib] (pads are left untouched).
__global__ void gen_kernel(KernelDev k, const double* pts, const double* nrm,
                           const int64_t* tpad, const GenItem* items, int64_t M, int64_t N) {
    const GenItem it = items[blockIdx.y];
    const int64_t rows = it.mode == 0 ? M : it.m;
    const int64_t cols = it.mode == 0 ? N : it.n;
    const int64_t total = rows * cols;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx % rows, j = idx / rows;
        if (it.mode == 0) {
            double v = (i < it.m && j < it.n) ? kernel_entry(k, pts, nrm, it.ib + i, it.jb + j) : 0.0;
            it.out[j * it.ld + i] = v;
        } else {
            int64_t row = tpad[it.ib + i] - tpad[it.ib];
            it.out[j * it.ld + row] = kernel_entry(k, pts, nrm, it.ib + i, it.jb + j);
        }
    }
}

// Sum of squares of `count` contiguous doubles per item, in two deterministic
// passes: fixed-size chunks, then the chunk partials in order.
__global__ void sumsq_partial_kernel(const SumItem* items, double* partial, int64_t chunk,
                                     int64_t nchunks) {
    __shared__ double red[256];
    const SumItem it = items[blockIdx.y];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = lo + chunk < it.count ? lo + chunk : it.count;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        double v = it.ptr[i];
        s += v * v;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * nchunks + blockIdx.x] = red[0];
}

__global__ void sumsq_final_kernel(const double* partial, int64_t nchunks, int nitems, double* out) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nitems) return;
    double s = 0.0;
    for (int64_t c = 0; c < nchunks; ++c) s += partial[(int64_t)b * nchunks + c];
    out[b] = s;
}

// SplitMix64 (Steele, Lea, Flood 2014): output k of the stream started at s is
// mix(s + k gamma).
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t GOLDEN_GAMMA = 0x9E3779B97F4A7C15ull;

// Rademacher sketch Omega (N x s, column-major, ld = N) of item b: entry
// (j, c) is the sign of output j s + c + 1 of the stream keyed by
// (seed, block uid, round); rows j >= n are 0.
__global__ void sketch_kernel(const SketchItem* items, int64_t N, int s, uint64_t seed) {
    const SketchItem it = items[blockIdx.y];
    const uint64_t a = mix64(seed + GOLDEN_GAMMA * (uint64_t)(it.uid + 1));
    const uint64_t key = mix64(a + GOLDEN_GAMMA * (uint64_t)(it.round + 1));
    const int64_t total = N * s;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = idx % N, c = idx / N;
        double v = 0.0;
        if (j < it.n) {
            uint64_t z = mix64(key + GOLDEN_GAMMA * (uint64_t)(j * s + c + 1));
            v = (z >> 63) ? -1.0 : 1.0;
        }
        it.out[c * N + j] = v;
    }
}

// Rank choice (Def. H_h(p, eps), Alg. 1): t(k) = extra + sum_{r >= k} sigma_r^2
// summed from the smallest term upward; rank = smallest k with t(k) <= thr.
// Randomized items are accepted when k + oversample <= s or s == min(m, n).
__global__ void rank_kernel(RankItem* items, int nitems, double eps2) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nitems) return;
    RankItem& it = items[b];
    it.norm2 = *it.norm2p;
    it.extra = it.extrap ? *it.extrap : 0.0;
    const double thr = eps2 * it.norm2;
    const int p = it.p;
    // t(k) is non-increasing in k, so scan k = p, p-1, ... while t(k) <= thr
    int k = -1;
    double tk = INFINITY, tprev = INFINITY;
    if (it.extra <= thr) {
        k = p;
        tk = it.extra;
        double acc = 0.0;
        for (int r = p - 1; r >= 0; --r) {
            acc += it.sigma[r] * it.sigma[r];
            double t = it.extra + acc;
            if (t <= thr) { k = r; tk = t; }
            else { tprev = t; break; }
        }
    }
    bool accept = true;
    if (it.sketch > 0) {
        if (k < 0 && it.sketch == it.pmin) { k = it.sketch; tk = it.extra; }
        accept = k >= 0 && (k + it.oversample <= it.sketch || it.sketch == it.pmin);
    }
    if (k < 0) k = p;
    double nb2 = 0.0;
    for (int r = 0; r < k; ++r) nb2 += it.sigma[r] * it.sigma[r];
    it.rank = k;
    it.accept = accept ? 1 : 0;
    it.tail = tk;
    it.tail_prev = k > 0 ? tprev : INFINITY;
    it.trunc2 = nb2;
}

// Write U (m x k) and V = W Sigma (n x k) of an accepted item into the fp64
// store in padded-row layout, after fixing signs so that the largest-|.|
// entry of each column of U (first index on ties) is positive.
__global__ void finalize_kernel(const FinItem* items, const int64_t* tpad) {
    __shared__ double bv[256];
    __shared__ int bi[256];
    const FinItem it = items[blockIdx.x];
    const int tid = threadIdx.x;
    for (int r = 0; r < it.k; ++r) {
        const double* u = it.U + (int64_t)r * it.ldu;
        double best = -1.0;
        int besti = 0x7fffffff;
        for (int i = tid; i < it.m; i += blockDim.x) {
            double a = fabs(u[i]);
            if (a > best) { best = a; besti = i; }
        }
        bv[tid] = best;
        bi[tid] = besti;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) {
                double o = bv[tid + w];
                int oi = bi[tid + w];
                if (o > bv[tid] || (o == bv[tid] && oi < bi[tid])) { bv[tid] = o; bi[tid] = oi; }
            }
            __syncthreads();
        }
        const double sgn = (bi[0] < it.m && u[bi[0]] < 0.0) ? -1.0 : 1.0;
        __syncthreads();
        double* uo = it.Uout + (int64_t)r * it.PI;
        const int64_t rb = tpad[it.ib];
        for (int i = tid; i < it.m; i += blockDim.x) uo[tpad[it.ib + i] - rb] = sgn * u[i];
        double* vo = it.Vout + (int64_t)r * it.PJ;
        const int64_t cb = tpad[it.jb];
        const double sr = sgn * it.sigma[r];
        for (int j = tid; j < it.n; j += blockDim.x)
            vo[tpad[it.jb + j] - cb] = sr * it.Vt[(int64_t)j * it.ldv + r];
    }
}

// Largest magnitude of each contiguous factor array.
__global__ void maxabs_kernel(const SumItem* items, double* out) {
    __shared__ double red[256];
    const SumItem it = items[blockIdx.x];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < it.count; i += blockDim.x) m = fmax(m, fabs(it.ptr[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Store 2^-e * src in format fmt (RNE), contiguous `count` elements.
__global__ void pack_kernel(const PackItem* items) {
    const PackItem it = items[blockIdx.y];
    const double sc = ldexp(1.0, -it.e);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < it.count;
         i += (int64_t)gridDim.x * blockDim.x) {
        double v = it.src[i] * sc;
        switch (it.fmt) {
            case HH_FMT_FP64: ((double*)it.dst)[i] = v; break;
            case HH_FMT_FP32: ((float*)it.dst)[i] = (float)v; break;
            case HH_FMT_FP16: ((uint16_t*)it.dst)[i] = f64_to_f16_rne(v); break;
            default: ((uint16_t*)it.dst)[i] = f64_to_bf16_rne(v); break;
        }
    }
}

// ------------------------------------------------------------ launchers
static inline unsigned grid_for(int64_t total, int64_t cap = 65535) {
    int64_t g = (total + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

void launch_gen(const KernelDev& k, const double* pts, const double* nrm, const int64_t* tpad,
                const GenItem* items, int nitems, int64_t M, int64_t N, int64_t max_total,
                hipStream_t s) {
    dim3 grid(grid_for(max_total, 8192), nitems);
    hipLaunchKernelGGL(gen_kernel, grid, dim3(256), 0, s, k, pts, nrm, tpad, items, M, N);
}

void launch_sumsq(const SumItem* items, int nitems, int64_t max_count, double* partial,
                  int64_t chunk, double* out, hipStream_t s) {
    int64_t nch = (max_count + chunk - 1) / chunk;
    if (nch < 1) nch = 1;
    hipLaunchKernelGGL(sumsq_partial_kernel, dim3((unsigned)nch, nitems), dim3(256), 0, s, items,
                       partial, chunk, nch);
    hipLaunchKernelGGL(sumsq_final_kernel, dim3((nitems + 255) / 256), dim3(256), 0, s, partial,
                       nch, nitems, out);
}

void launch_sketch(const SketchItem* items, int nitems, int64_t N, int sk, uint64_t seed,
                   hipStream_t s) {
    dim3 grid(grid_for(N * sk, 4096), nitems);
    hipLaunchKernelGGL(sketch_kernel, grid, dim3(256), 0, s, items, N, sk, seed);
}

void launch_rank(RankItem* items, int nitems, double eps2, hipStream_t s) {
    hipLaunchKernelGGL(rank_kernel, dim3((nitems + 63) / 64), dim3(64), 0, s, items, nitems, eps2);
}

void launch_finalize(const FinItem* items, int nitems, const int64_t* tpad, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(nitems), dim3(256), 0, s, items, tpad);
}

void launch_maxabs(const SumItem* items, int nitems, double* out, hipStream_t s) {
    hipLaunchKernelGGL(maxabs_kernel, dim3(nitems), dim3(256), 0, s, items, out);
}

void launch_pack(const PackItem* items, int nitems, int64_t max_count, hipStream_t s) {
    dim3 grid(grid_for(max_count, 2048), nitems);
    hipLaunchKernelGGL(pack_kernel, grid, dim3(256), 0, s, items);
}

}  // namespace hh
