// Device kernels of the construction stage (Alg. 1, Alg. 5, Alg. 3):
// kernel-matrix entries, Frobenius sums, Rademacher sketches, rank choice,
// factor finalisation and rounding into the storage formats.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hh_build.h"

namespace hh {

static inline unsigned grid_for(int64_t total, int64_t cap = 65535) {
    int64_t g = (total + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

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

// q43 (the 8-bit row of Table tab:precisions): sign, 4 exponent bits with
// bias 7, 3 fraction bits; normal exponents -6..7, gradual underflow below
// 2^-6 (spacing 2^-9), largest finite value 240; the same bit patterns as OCP
// fp8 e4m3 below 256. RNE straight from fp64. Magnitudes that round beyond
// 240 saturate to it (factors are scaled so that their largest entry lies in
// [64, 128), so none does).
__host__ __device__ uint8_t f64_to_q43_rne(double x) {
    const uint64_t bits = __builtin_bit_cast(uint64_t, x);
    const uint8_t sign = (uint8_t)((bits >> 56) & 0x80u);
    const int ex = (int)((bits >> 52) & 0x7FF);
    const uint64_t man = bits & ((1ull << 52) - 1);
    if (ex == 0x7FF) return sign | 0x77u;
    if (ex == 0) return sign;
    const int e = ex - 1023;
    if (e > 8) return sign | 0x77u;
    const uint64_t M = man | (1ull << 52);          // value = M 2^(e - 52)
    const int ue = (e > -6 ? e : -6) - 3;           // exponent of the spacing
    const int shift = 52 + ue - e;                  // >= 49
    if (shift >= 64) return sign;
    uint64_t q = M >> shift;
    const uint64_t rem = M & ((1ull << shift) - 1);
    const uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    // normal: q in [8, 16] times 2^(e - 3); a carry to 16 moves to the next binade
    uint32_t out = e >= -6 ? (uint32_t)((e + 7) << 3) + (uint32_t)q - 8u : (uint32_t)q;
    if (out > 0x77u) out = 0x77u;
    return sign | (uint8_t)out;
}

__host__ __device__ double q43_to_f64(uint8_t c) {
    const int field = (c >> 3) & 15, frac = c & 7;
    const double v = field ? std::ldexp((double)(8 + frac), field - 10) : std::ldexp((double)frac, -9);
    return (c & 0x80u) ? -v : v;
}

// Continuum storage: t fraction bits (7 <= t <= 23) behind an 8-bit exponent
// with the exponent range of fp32 (gradual underflow below 2^-126), sign
// first: a (9 + t)-bit code equal to the top 9 + t bits of the fp32 encoding of
// the rounded value (every such value is an fp32 number). t = 7 is bf16.
__host__ __device__ uint32_t f64_to_cont_rne(double x, int t) {
    const uint64_t bits = __builtin_bit_cast(uint64_t, x);
    const uint32_t sign = (uint32_t)(bits >> 63) << (8 + t);
    const uint32_t inf = 0xFFu << t;
    int ex = (int)((bits >> 52) & 0x7FF);
    uint64_t man = bits & ((1ull << 52) - 1);
    if (ex == 0x7FF) return sign | inf | (man ? (1u << (t - 1)) : 0u);
    if (ex == 0) return sign;
    int e = ex - 1023;
    if (e > 127) return sign | inf;
    uint64_t M = man | (1ull << 52);
    int ue = (e > -126 ? e : -126) - t;             // exponent of the ulp at |x|
    int shift = 52 + ue - e;                        // >= 29
    if (shift >= 64) return sign;
    uint64_t q = M >> shift;
    uint64_t rem = M & ((1ull << shift) - 1);
    uint64_t half = 1ull << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    uint32_t out = e >= -126 ? ((uint32_t)(e + 127) << t) + (uint32_t)q - (1u << t) : (uint32_t)q;
    if (out >= inf) out = inf;
    return sign | out;
}

__host__ __device__ double cont_to_f64(uint32_t code, int t) {
    return (double)__builtin_bit_cast(float, code << (23 - t));
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

// Write U (m x k) and V (n x k) of an accepted item into the fp64 store in
// padded-row layout, after fixing signs so that the largest-|.| entry of each
// column of U (first index on ties) is positive.
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
        if (it.v_rows) {
            const double sr = sgn * it.sigma[r];
            for (int j = tid; j < it.n; j += blockDim.x)
                vo[tpad[it.jb + j] - cb] = sr * it.V[(int64_t)j * it.ldv + r];
        } else {
            const double* v = it.V + (int64_t)r * it.ldv;
            for (int j = tid; j < it.n; j += blockDim.x) vo[tpad[it.jb + j] - cb] = sgn * v[j];
        }
    }
}

// Householder QR of one m x n panel per workgroup (column-major, leading
// dimension ld, items strideA / strideT apart), in LAPACK geqrf layout: R on
// and above the diagonal, the reflectors v (v_j = 1 implied) below it, tau[j];
// A = H_1 ... H_n R with H_j = I - tau_j v v^T. Reflector j follows dlarfg:
// beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta, v = x / (alpha - beta);
// tau = 0 when the part below the diagonal is already zero. Trailing columns
// are updated in chunks of 32 with one block-wide reduction per chunk.
__global__ __launch_bounds__(256) void house_qr_kernel(double* A, int64_t ld, int64_t strideA,
                                                       double* tau, int64_t strideT, int64_t m,
                                                       int n) {
    __shared__ double red[4][33];
    __shared__ double bc[33];
    double* a = A + (int64_t)blockIdx.x * strideA;
    double* tj = tau + (int64_t)blockIdx.x * strideT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int jmax = (int)(n < m ? n : m);
    for (int j = 0; j < jmax; ++j) {
        double* col = a + (int64_t)j * ld;
        double ss = 0.0;
        for (int64_t i = j + 1 + tid; i < m; i += 256) ss += col[i] * col[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
        if (lane == 0) red[wave][0] = ss;
        __syncthreads();
        const double sigma = red[0][0] + red[1][0] + red[2][0] + red[3][0];
        const double alpha = col[j];
        double t = 0.0, beta = alpha, scal = 0.0;
        if (sigma != 0.0) {
            const double nrm = sqrt(alpha * alpha + sigma);
            beta = alpha >= 0.0 ? -nrm : nrm;
            t = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        __syncthreads();
        if (t != 0.0)
            for (int64_t i = j + 1 + tid; i < m; i += 256) col[i] *= scal;
        if (tid == 0) {
            tj[j] = t;
            col[j] = beta;
        }
        __syncthreads();
        if (t == 0.0) continue;
        // trailing update: w_c = v^T a_c, a_c -= t v w_c for c = j+1 .. n-1
        for (int c0 = j + 1; c0 < n; c0 += 32) {
            const int nc = n - c0 < 32 ? n - c0 : 32;
            double w[32];
#pragma unroll
            for (int c = 0; c < 32; ++c) w[c] = 0.0;
            for (int64_t i = j + tid; i < m; i += 256) {
                const double v = i == j ? 1.0 : col[i];
#pragma unroll
                for (int c = 0; c < 32; ++c)
                    if (c < nc) w[c] += v * a[(int64_t)(c0 + c) * ld + i];
            }
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                double x = w[c];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
                if (lane == 0) red[wave][c] = x;
            }
            __syncthreads();
            if (tid < nc) bc[tid] = t * (red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid]);
            __syncthreads();
            for (int64_t i = j + tid; i < m; i += 256) {
                const double v = i == j ? 1.0 : col[i];
                for (int c = 0; c < nc; ++c) a[(int64_t)(c0 + c) * ld + i] -= v * bc[c];
            }
            __syncthreads();
        }
    }
}

// Reduce-scatter of NV (a power of two <= 64) values across a wavefront: the
// first log2(NV) butterfly steps exchange half of the values still held, so
// that after them each lane keeps one partial sum; the remaining steps add the
// lanes that hold the same value. Returns the wave total of value
// lane / (64 / NV). v is consumed.
template <int C, int NV>
__device__ inline void rs_step(double (&v)[NV], int lane) {
    if constexpr (C > 1) {
        constexpr int half = C / 2;
        constexpr int off = 32 * C / NV;
        const bool hi = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const double send = hi ? v[i] : v[i + half];
            const double keep = hi ? v[i + half] : v[i];
            v[i] = keep + __shfl_xor(send, off, 64);
        }
        rs_step<half, NV>(v, lane);
    }
}

template <int NV>
__device__ inline double wave_rs(double (&v)[NV], int lane) {
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV: power of two <= 64");
    rs_step<NV, NV>(v, lane);
    double x = v[0];
#pragma unroll
    for (int off = 32 / NV; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Sums of NV per-thread values over a block of NW waves into out[0 .. NV), in
// a fixed order (wave butterflies, then the waves in order).
template <int NV, int NW>
__device__ inline void block_sum(double (&v)[NV], double* red, double* out, int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    const double x = wave_rs<NV>(v, lane);
    constexpr int SH = 64 / NV;
    if ((lane & (SH - 1)) == 0) red[wave * NV + lane / SH] = x;
    __syncthreads();
    if (tid < NV) {
        double t = red[tid];
#pragma unroll
        for (int w = 1; w < NW; ++w) t += red[w * NV + tid];
        out[tid] = t;
    }
    __syncthreads();
}

// The same factorization as house_qr_kernel (geqrf layout, the same reflector
// definition) for m <= 64 NW RPT rows and n <= m columns. Panels of HQ_PB
// columns are held in registers (thread t owns rows t + 64 NW q, q < RPT) and
// factored there; the trailing columns are then updated once per panel with the compact
// WY form I - V T^T V^T of the panel's reflectors (T upper triangular from
// V^T V and tau, as in LAPACK's dlarft), HQ_G columns per block reduction.
constexpr int HQ_PB = 8;
constexpr int HQ_G = 4;
constexpr int64_t HOUSE_REG_MAX = 4096;   // rows handled by house_qr_reg_kernel
template <int RPT, int NW>
__global__ __launch_bounds__(64 * NW) void house_qr_reg_kernel(double* A, int64_t ld,
                                                               int64_t strideA, double* tau,
                                                               int64_t strideT, int m, int n) {
    constexpr int NTH = 64 * NW;
    __shared__ double red[NW * 64];
    __shared__ double out[64];
    __shared__ double T[HQ_PB * HQ_PB];
    __shared__ double W2[HQ_PB * HQ_G];
    __shared__ double tl[HQ_PB];
    double* a = A + (int64_t)blockIdx.x * strideA;
    double* tj = tau + (int64_t)blockIdx.x * strideT;
    const int tid = threadIdx.x;
    for (int c0 = 0; c0 < n; c0 += HQ_PB) {
        const int pb = n - c0 < HQ_PB ? n - c0 : HQ_PB;
        double P[RPT][HQ_PB];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = tid + NTH * q;
#pragma unroll
            for (int k = 0; k < HQ_PB; ++k)
                P[q][k] = (i >= c0 && i < m && k < pb) ? a[(int64_t)(c0 + k) * ld + i] : 0.0;
        }
        // factor the panel
#pragma unroll
        for (int k = 0; k < HQ_PB; ++k) {
            if (k >= pb) break;
            const int j = c0 + k;
            double s2[2] = {0.0, 0.0};
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = tid + NTH * q;
                if (i > j && i < m) s2[0] += P[q][k] * P[q][k];
                if (i == j) s2[1] = P[q][k];
            }
            block_sum<2, NW>(s2, red, out, tid);
            const double sigma = out[0], alpha = out[1];
            double t = 0.0, beta = alpha, scal = 0.0;
            if (sigma != 0.0) {
                const double nrm = sqrt(alpha * alpha + sigma);
                beta = alpha >= 0.0 ? -nrm : nrm;
                t = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = tid + NTH * q;
                if (i > j && i < m && t != 0.0) P[q][k] *= scal;
                if (i == j) P[q][k] = beta;
            }
            if (tid == 0) {
                tj[j] = t;
                tl[k] = t;
            }
            if (t == 0.0 || k + 1 >= pb) continue;
            double w[HQ_PB];
#pragma unroll
            for (int kk = 0; kk < HQ_PB; ++kk) w[kk] = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = tid + NTH * q;
                const double vi = i == j ? 1.0 : (i > j && i < m ? P[q][k] : 0.0);
#pragma unroll
                for (int kk = k + 1; kk < HQ_PB; ++kk) w[kk] += vi * P[q][kk];
            }
            block_sum<HQ_PB, NW>(w, red, out, tid);
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = tid + NTH * q;
                const double vi = i == j ? 1.0 : (i > j && i < m ? P[q][k] : 0.0);
#pragma unroll
                for (int kk = k + 1; kk < HQ_PB; ++kk) P[q][kk] -= t * vi * out[kk];
            }
        }
        // write the panel back (rows >= c0) and turn P into the reflectors V
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int i = tid + NTH * q;
#pragma unroll
            for (int k = 0; k < HQ_PB; ++k) {
                if (i >= c0 && i < m && k < pb) a[(int64_t)(c0 + k) * ld + i] = P[q][k];
                const int j = c0 + k;
                P[q][k] = (k < pb && i < m) ? (i == j ? 1.0 : (i > j ? P[q][k] : 0.0)) : 0.0;
            }
        }
        if (c0 + pb >= n) break;
        // T from the strictly upper part of V^T V (28 pairs)
        double g[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) g[c] = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            int c = 0;
#pragma unroll
            for (int x = 0; x < HQ_PB; ++x)
#pragma unroll
                for (int y = x + 1; y < HQ_PB; ++y) g[c++] += P[q][x] * P[q][y];
        }
        block_sum<32, NW>(g, red, out, tid);
        if (tid == 0) {
            // T[x + HQ_PB y] = T(x, y), upper triangular
            for (int i = 0; i < HQ_PB * HQ_PB; ++i) T[i] = 0.0;
            for (int y = 0; y < pb; ++y) {
                T[y + HQ_PB * y] = tl[y];
                for (int x = 0; x < y; ++x) {
                    double z = 0.0;
                    for (int c = x; c < y; ++c) {
                        const int gi = c * (2 * HQ_PB - c - 1) / 2 + (y - c - 1);  // pair (c, y)
                        z += T[x + HQ_PB * c] * out[gi];
                    }
                    T[x + HQ_PB * y] = -tl[y] * z;
                }
            }
        }
        __syncthreads();
        // trailing columns: C <- C - V (T^T (V^T C))
        for (int g0 = c0 + pb; g0 < n; g0 += HQ_G) {
            const int gw = n - g0 < HQ_G ? n - g0 : HQ_G;
            double wv[HQ_PB * HQ_G];
#pragma unroll
            for (int c = 0; c < HQ_PB * HQ_G; ++c) wv[c] = 0.0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = tid + NTH * q;
                if (i < c0 || i >= m) continue;
#pragma unroll
                for (int c = 0; c < HQ_G; ++c) {
                    if (c >= gw) break;
                    const double x = a[(int64_t)(g0 + c) * ld + i];
#pragma unroll
                    for (int y = 0; y < HQ_PB; ++y) wv[y * HQ_G + c] += P[q][y] * x;
                }
            }
            block_sum<HQ_PB * HQ_G, NW>(wv, red, out, tid);
            if (tid < HQ_PB * HQ_G) {
                const int y = tid / HQ_G, c = tid % HQ_G;
                double z = 0.0;
                for (int x = 0; x <= y; ++x) z += T[x + HQ_PB * y] * out[x * HQ_G + c];
                W2[tid] = z;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int i = tid + NTH * q;
                if (i < c0 || i >= m) continue;
#pragma unroll
                for (int c = 0; c < HQ_G; ++c) {
                    if (c >= gw) break;
                    double* px = a + (int64_t)(g0 + c) * ld + i;
                    double x = *px;
#pragma unroll
                    for (int y = 0; y < HQ_PB; ++y) x -= P[q][y] * W2[y * HQ_G + c];
                    *px = x;
                }
            }
        }
    }
}

void launch_house_qr(double* A, int64_t ld, int64_t strideA, double* tau, int64_t strideT,
                     int64_t m, int n, int nitems, hipStream_t st) {
    if (n <= m && m <= HOUSE_REG_MAX) {
        const int mi = (int)m;
        if (m <= 256)
            hipLaunchKernelGGL((house_qr_reg_kernel<1, 4>), dim3(nitems), dim3(256), 0, st, A, ld,
                               strideA, tau, strideT, mi, n);
        else if (m <= 512)
            hipLaunchKernelGGL((house_qr_reg_kernel<2, 4>), dim3(nitems), dim3(256), 0, st, A, ld,
                               strideA, tau, strideT, mi, n);
        else if (m <= 1024)
            hipLaunchKernelGGL((house_qr_reg_kernel<4, 4>), dim3(nitems), dim3(256), 0, st, A, ld,
                               strideA, tau, strideT, mi, n);
        else if (m <= 2048)
            hipLaunchKernelGGL((house_qr_reg_kernel<8, 4>), dim3(nitems), dim3(256), 0, st, A, ld,
                               strideA, tau, strideT, mi, n);
        else
            hipLaunchKernelGGL((house_qr_reg_kernel<8, 8>), dim3(nitems), dim3(512), 0, st, A, ld,
                               strideA, tau, strideT, mi, n);
        return;
    }
    hipLaunchKernelGGL(house_qr_kernel, dim3(nitems), dim3(256), 0, st, A, ld, strideA, tau,
                       strideT, m, n);
}

// Panel reflectors -> unit lower trapezoidal V (m x nb, contiguous, zero column
// where tau = 0) and the identity in T (nb x nb), for the compact-WY update of
// the trailing columns in a blocked QR.
__global__ void panel_v_kernel(const double* A, int64_t ld, int64_t strideA, const double* tau,
                               int64_t strideT, double* V, double* T, int64_t m, int nb) {
    const double* a = A + (int64_t)blockIdx.y * strideA;
    const double* tj = tau + (int64_t)blockIdx.y * strideT;
    double* v = V + (int64_t)blockIdx.y * m * nb;
    double* t = T + (int64_t)blockIdx.y * nb * nb;
    const int64_t total = m * nb;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % m, j = idx / m;
        double x = i > j ? a[j * ld + i] : (i == j ? 1.0 : 0.0);
        if (tj[j] == 0.0) x = 0.0;
        v[idx] = x;
        if (i < nb) t[i + j * nb] = i == j ? 1.0 : 0.0;
    }
}

// Tinv = diag(1/tau) + strict upper part of G for a panel (batch strides).
__global__ void panel_tinv_kernel(const double* G, const double* tau, int64_t strideT,
                                  double* Tinv, int nb) {
    const double* g = G + (int64_t)blockIdx.x * nb * nb;
    const double* tj = tau + (int64_t)blockIdx.x * strideT;
    double* ti = Tinv + (int64_t)blockIdx.x * nb * nb;
    for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
        const int i = idx % nb, j = idx / nb;
        double x = 0.0;
        if (i < j) x = g[idx];
        else if (i == j) x = tj[j] != 0.0 ? 1.0 / tj[j] : 1.0;
        ti[idx] = x;
    }
}

void launch_panel_v(const double* A, int64_t ld, int64_t strideA, const double* tau,
                    int64_t strideT, double* V, double* T, int64_t m, int nb, int nitems,
                    hipStream_t st) {
    dim3 grid(grid_for(m * nb, 1024), nitems);
    hipLaunchKernelGGL(panel_v_kernel, grid, dim3(256), 0, st, A, ld, strideA, tau, strideT, V, T,
                       m, nb);
}

void launch_panel_tinv(const double* G, const double* tau, int64_t strideT, double* Tinv, int nb,
                       int nitems, hipStream_t st) {
    hipLaunchKernelGGL(panel_tinv_kernel, dim3(nitems), dim3(256), 0, st, G, tau, strideT, Tinv, nb);
}

// geqrf output -> unit lower trapezoidal reflectors Vm (a zero column where
// tau = 0, i.e. where the reflector is the identity), the R factor, [I; 0]
// into Q and the identity into T.
__global__ void qr_extract_kernel(const QrItem* items, int64_t rows, int s) {
    const QrItem it = items[blockIdx.y];
    const int64_t total = rows * s;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % rows, j = idx / rows;
        double v = i > j ? it.A[idx] : (i == j ? 1.0 : 0.0);
        if (it.tau[j] == 0.0) v = 0.0;
        it.Vm[idx] = v;
        it.Q[idx] = i == j ? 1.0 : 0.0;
        if (i < s) {
            if (it.R) it.R[i + j * s] = i <= j ? it.A[idx] : 0.0;
            it.T[i + j * s] = i == j ? 1.0 : 0.0;
        }
    }
}

// T^-1 = diag(1/tau) + strictly upper part of V^T V, so that
// H_1 ... H_s = I - V T V^T (compact WY form of the reflectors).
__global__ void qr_tinv_kernel(const QrItem* items, int s) {
    const QrItem it = items[blockIdx.y];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < s * s; idx += gridDim.x * blockDim.x) {
        const int i = idx % s, j = idx / s;
        double v = 0.0;
        if (i < j) v = it.G[idx];
        else if (i == j) v = it.tau[j] != 0.0 ? 1.0 / it.tau[j] : 1.0;
        it.Tinv[idx] = v;
    }
}

// One-sided (Hestenes) Jacobi SVD of an s x s matrix, s <= 64, in LDS.
// Pairs follow the round-robin (circle) ordering; 8 lanes per pair. Columns of
// A are rotated until pairwise orthogonal to 1e-15 relative (at most 40
// sweeps), J accumulates the rotations, and columns are sorted by norm.
constexpr int JAC_MAX = 64;
__global__ __launch_bounds__(256) void jacobi_kernel(const JacItem* items, int s) {
    __shared__ double A[JAC_MAX * JAC_MAX];
    __shared__ double J[JAC_MAX * JAC_MAX];
    __shared__ double sig[JAC_MAX];
    __shared__ int order[JAC_MAX];
    __shared__ int rotated;
    const JacItem it = items[blockIdx.x];
    const int tid = threadIdx.x;
    for (int i = tid; i < s * s; i += 256) {
        A[i] = it.A[i];
        J[i] = (i % s == i / s) ? 1.0 : 0.0;
    }
    const int se = s + (s & 1);          // even number of players (one dummy when s is odd)
    const int npairs = se / 2;
    const int pair = tid >> 3, lane8 = tid & 7;
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int r = 0; r < se - 1; ++r) {
            int p = -1, q = -1;
            if (pair < npairs) {
                if (pair == 0) {
                    p = 0;
                    q = (r % (se - 1)) + 1;
                } else {
                    p = ((pair + r) % (se - 1)) + 1;
                    q = ((se - 1 - pair + r) % (se - 1)) + 1;
                }
                if (p > q) { int t = p; p = q; q = t; }
            }
            const bool live = pair < npairs && q < s;
            double al = 0.0, be = 0.0, ga = 0.0;
            if (live)
                for (int i = lane8; i < s; i += 8) {
                    const double a = A[i + p * s], b = A[i + q * s];
                    al += a * a;
                    be += b * b;
                    ga += a * b;
                }
#pragma unroll
            for (int off = 4; off > 0; off >>= 1) {
                al += __shfl_xor(al, off, 8);
                be += __shfl_xor(be, off, 8);
                ga += __shfl_xor(ga, off, 8);
            }
            if (live && ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                for (int i = lane8; i < s; i += 8) {
                    const double a = A[i + p * s], b = A[i + q * s];
                    A[i + p * s] = c * a - sn * b;
                    A[i + q * s] = sn * a + c * b;
                    const double x = J[i + p * s], y = J[i + q * s];
                    J[i + p * s] = c * x - sn * y;
                    J[i + q * s] = sn * x + c * y;
                }
                if (lane8 == 0) rotated = 1;
            }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
    if (tid < s) {
        double a = 0.0;
        for (int i = 0; i < s; ++i) a += A[i + tid * s] * A[i + tid * s];
        sig[tid] = sqrt(a);
    }
    __syncthreads();
    if (tid == 0) {
        for (int i = 0; i < s; ++i) order[i] = i;
        for (int i = 0; i < s; ++i) {      // selection sort, decreasing; ties keep index order
            int b = i;
            for (int j = i + 1; j < s; ++j)
                if (sig[order[j]] > sig[order[b]]) b = j;
            int t = order[i]; order[i] = order[b]; order[b] = t;
        }
    }
    __syncthreads();
    for (int idx = tid; idx < s * s; idx += 256) {
        const int i = idx % s, r = idx / s, c = order[r];
        it.A[idx] = A[i + c * s];
        it.J[idx] = J[i + c * s];
    }
    if (tid < s) it.sigma[tid] = sig[order[tid]];
}

// One-sided Jacobi SVD for 64 < s <= 128 with the columns in registers: 512
// threads form 64 slot pairs of 8 lanes; each lane keeps 16 rows (i = lane +
// 8 r) of the two columns of A and of J its pair holds. Every step rotates
// each pair, then the columns move one seat along the round-robin circle
// (seat 0 fixed) through LDS, so every pair of columns meets once per sweep.
// Same rotation, stopping rule and sorted output as the s <= 64 kernel.
__global__ __launch_bounds__(512) void jacobi128_kernel(const JacItem* items, int s) {
    __shared__ double buf[128 * 128];
    __shared__ double sig[128];
    __shared__ int order[128];
    __shared__ int rotated;
    const JacItem it = items[blockIdx.x];
    const int tid = threadIdx.x, g = tid >> 3, l = tid & 7;
    const int S = s + (s & 1), P = S / 2;
    const bool active = g < P;
    double at[16], ab[16], jt[16], jb[16];
    {
        const int ct = g, cb = S - 1 - g;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = l + 8 * r;
            at[r] = (active && i < s && ct < s) ? it.A[i + ct * s] : 0.0;
            ab[r] = (active && i < s && cb < s) ? it.A[i + cb * s] : 0.0;
            jt[r] = (active && i == ct && ct < s) ? 1.0 : 0.0;
            jb[r] = (active && i == cb && cb < s) ? 1.0 : 0.0;
        }
    }
    // seat that feeds my top / bottom slot after a step (slot index 2g = top, 2g+1 = bottom)
    const int src_top = g == 0 ? 0 : (g == 1 ? 1 : 2 * (g - 1));
    const int src_bot = g == P - 1 ? 2 * (P - 1) : 2 * (g + 1) + 1;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int step = 0; step < S - 1; ++step) {
            double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                al += at[r] * at[r];
                be += ab[r] * ab[r];
                ga += at[r] * ab[r];
            }
#pragma unroll
            for (int off = 4; off > 0; off >>= 1) {
                al += __shfl_xor(al, off, 8);
                be += __shfl_xor(be, off, 8);
                ga += __shfl_xor(ga, off, 8);
            }
            if (active && ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const double a = at[r], b = ab[r];
                    at[r] = c * a - sn * b;
                    ab[r] = sn * a + c * b;
                    const double x = jt[r], y = jb[r];
                    jt[r] = c * x - sn * y;
                    jb[r] = sn * x + c * y;
                }
                if (l == 0) rotated = 1;
            }
            // move the columns one seat along the circle
            if (active)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    buf[(2 * g) * 128 + l + 8 * r] = at[r];
                    buf[(2 * g + 1) * 128 + l + 8 * r] = ab[r];
                }
            __syncthreads();
            if (active)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    at[r] = buf[src_top * 128 + l + 8 * r];
                    ab[r] = buf[src_bot * 128 + l + 8 * r];
                }
            __syncthreads();
            if (active)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    buf[(2 * g) * 128 + l + 8 * r] = jt[r];
                    buf[(2 * g + 1) * 128 + l + 8 * r] = jb[r];
                }
            __syncthreads();
            if (active)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    jt[r] = buf[src_top * 128 + l + 8 * r];
                    jb[r] = buf[src_bot * 128 + l + 8 * r];
                }
            __syncthreads();
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
    // norms per slot, rank of each slot by decreasing norm (ties: lower slot first)
    if (active)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            buf[(2 * g) * 128 + l + 8 * r] = at[r];
            buf[(2 * g + 1) * 128 + l + 8 * r] = ab[r];
        }
    __syncthreads();
    if (tid < S) {
        double a = 0.0;
        for (int i = 0; i < s; ++i) a += buf[tid * 128 + i] * buf[tid * 128 + i];
        sig[tid] = sqrt(a);
    }
    __syncthreads();
    if (tid < S) {
        int rank = 0;
        for (int u = 0; u < S; ++u)
            if (sig[u] > sig[tid] || (sig[u] == sig[tid] && u < tid)) ++rank;
        order[rank] = tid;
    }
    __syncthreads();
    for (int idx = tid; idx < s * s; idx += 512) {
        const int i = idx % s, r = idx / s;
        it.A[idx] = buf[order[r] * 128 + i];
    }
    if (tid < s) it.sigma[tid] = sig[order[tid]];
    __syncthreads();
    if (active)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            buf[(2 * g) * 128 + l + 8 * r] = jt[r];
            buf[(2 * g + 1) * 128 + l + 8 * r] = jb[r];
        }
    __syncthreads();
    for (int idx = tid; idx < s * s; idx += 512) {
        const int i = idx % s, r = idx / s;
        it.J[idx] = buf[order[r] * 128 + i];
    }
}

void launch_jacobi128(const JacItem* items, int nitems, int s, hipStream_t st) {
    hipLaunchKernelGGL(jacobi128_kernel, dim3(nitems), dim3(512), 0, st, items, s);
}

// One-sided Jacobi SVD for 128 < s <= 512 with the matrix in global memory.
// Each item works on [A; J] (2s rows, sp >= s columns padded with zero columns,
// column-major in work): the columns form nb = sp / b blocks of b (16 up to
// s = 256, else 8); a sweep visits every pair of blocks once (round-robin), and
// each visit loads the two blocks into LDS and rotates every pair of their 2b
// columns once (round-robin again, one wave per column pair, b waves). Same
// rotation as the kernels above; a pair is skipped when
// |a_p^T a_q| <= tol ||a_p|| ||a_q|| with tol = s 2^-53 (the rounding level of
// an inner product of length s: below it rotations only chase rounding noise),
// and the sweeps stop when one rotates nothing (at most 40). Zero (padding)
// columns never rotate. Output sorted as in the kernels above.
constexpr int JT_TILE = 32 * 528;     // 2b columns x (2s + 16) rows, b s = 4096
__device__ inline void rr_pair(int n, int round, int k, int& p, int& q) {
    // circle method for n (even) players: player n - 1 fixed
    if (k == 0) {
        p = round;
        q = n - 1;
    } else {
        p = (round + k) % (n - 1);
        q = (round - k + (n - 1)) % (n - 1);
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

template <int B>
__global__ __launch_bounds__(64 * B) void jacobi_tiled_kernel(const JacItem* items, double* work,
                                                              int s, int sp) {
    constexpr int NTH = 64 * B, N2 = 2 * B;
    __shared__ double tile[JT_TILE];
    __shared__ double sig[512];
    __shared__ int order[512];
    __shared__ int rotated;
    const JacItem it = items[blockIdx.x];
    const int tid = threadIdx.x;
    const int R = 2 * s, ldt = R + 16, nb = sp / B;
    const int pr = tid >> 6, ln = tid & 63;
    double* w = work + (int64_t)blockIdx.x * R * sp;
    for (int64_t idx = tid; idx < (int64_t)R * sp; idx += NTH) {
        const int i = (int)(idx % R), c = (int)(idx / R);
        double v = 0.0;
        if (c < s) v = i < s ? it.A[i + (int64_t)c * s] : (i - s == c ? 1.0 : 0.0);
        w[idx] = v;
    }
    const double tol = (double)s * 0x1p-53;
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int ro = 0; ro < nb - 1; ++ro) {
            for (int k = 0; k < nb / 2; ++k) {
                int B1, B2;
                rr_pair(nb, ro, k, B1, B2);
                for (int idx = tid; idx < N2 * R; idx += NTH) {
                    const int i = idx % R, c = idx / R;
                    const int gc = c < B ? B1 * B + c : B2 * B + (c - B);
                    tile[c * ldt + i] = w[(int64_t)gc * R + i];
                }
                __syncthreads();
                for (int r = 0; r < N2 - 1; ++r) {
                    int p, q;
                    rr_pair(N2, r, pr, p, q);
                    double* up = tile + p * ldt;
                    double* uq = tile + q * ldt;
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll 4
                    for (int i = ln; i < s; i += 64) {
                        const double x = up[i], y = uq[i];
                        al += x * x;
                        be += y * y;
                        ga += x * y;
                    }
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) {
                        al += __shfl_xor(al, off, 64);
                        be += __shfl_xor(be, off, 64);
                        ga += __shfl_xor(ga, off, 64);
                    }
                    if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                        const double zeta = (be - al) / (2.0 * ga);
                        const double t =
                            (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll 4
                        for (int i = ln; i < R; i += 64) {
                            const double x = up[i], y = uq[i];
                            up[i] = c * x - sn * y;
                            uq[i] = sn * x + c * y;
                        }
                        if (ln == 0) rotated = 1;
                    }
                    __syncthreads();
                }
                for (int idx = tid; idx < N2 * R; idx += NTH) {
                    const int i = idx % R, c = idx / R;
                    const int gc = c < B ? B1 * B + c : B2 * B + (c - B);
                    w[(int64_t)gc * R + i] = tile[c * ldt + i];
                }
                __syncthreads();
            }
        }
        const int any = rotated;
        __syncthreads();
        if (!any) break;
    }
    for (int c = tid; c < sp; c += NTH) {
        double a = 0.0;
        const double* col = w + (int64_t)c * R;
        for (int i = 0; i < s; ++i) a += col[i] * col[i];
        sig[c] = sqrt(a);
    }
    __syncthreads();
    for (int c = tid; c < sp; c += NTH) {
        int rank = 0;
        for (int u = 0; u < sp; ++u)
            if (sig[u] > sig[c] || (sig[u] == sig[c] && u < c)) ++rank;
        order[rank] = c;
    }
    __syncthreads();
    for (int64_t idx = tid; idx < (int64_t)s * s; idx += NTH) {
        const int i = (int)(idx % s), r = (int)(idx / s);
        const double* col = w + (int64_t)order[r] * R;
        it.A[idx] = col[i];
        it.J[idx] = col[s + i];
    }
    for (int r = tid; r < s; r += NTH) it.sigma[r] = sig[order[r]];
}

int jacobi_tiled_width(int s) { return s <= 256 ? 16 : 8; }
int jacobi_tiled_cols(int s) {
    const int b2 = 2 * jacobi_tiled_width(s);
    return (s + b2 - 1) / b2 * b2;
}

void launch_jacobi_tiled(const JacItem* items, double* work, int nitems, int s, hipStream_t st) {
    if (jacobi_tiled_width(s) == 16)
        hipLaunchKernelGGL(jacobi_tiled_kernel<16>, dim3(nitems), dim3(1024), 0, st, items, work, s,
                           jacobi_tiled_cols(s));
    else
        hipLaunchKernelGGL(jacobi_tiled_kernel<8>, dim3(nitems), dim3(512), 0, st, items, work, s,
                           jacobi_tiled_cols(s));
}

// rocSOLVER SVD R = U S V^T of a square s x s matrix -> the Jacobi outputs:
// A <- U S (columns sigma_r u_r), J <- V.
__global__ void svd_to_jac_kernel(const JacItem* items, const double* U, const double* Vt, int s) {
    const JacItem it = items[blockIdx.y];
    const double* u = U + (int64_t)blockIdx.y * s * s;
    const double* vt = Vt + (int64_t)blockIdx.y * s * s;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < s * s; idx += gridDim.x * blockDim.x) {
        const int i = idx % s, r = idx / s;
        it.A[idx] = u[idx] * it.sigma[r];
        it.J[idx] = vt[r + i * s];
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
            case HH_FMT_Q43: ((uint8_t*)it.dst)[i] = f64_to_q43_rne(v); break;
            default: ((uint16_t*)it.dst)[i] = f64_to_bf16_rne(v); break;
        }
    }
}

// One thread per output dword: the entries overlapping bits [32 j, 32 j + 32)
// of column c, each rounded to t fraction bits (entries past P are zero).
__global__ void pack_cont_kernel(const ContPackItem* items) {
    const ContPackItem it = items[blockIdx.y];
    const int w = 9 + it.t;
    const int64_t total = (int64_t)it.k * it.cdw;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = q / it.cdw, j = q - c * it.cdw;
        const int64_t b0 = 32 * j;
        const int64_t i0 = b0 / w, i1 = (b0 + 31) / w;
        uint64_t acc = 0;
        for (int64_t i = i0; i <= i1 && i < it.P; ++i) {
            const uint64_t code = f64_to_cont_rne(it.src[c * it.P + i], it.t);
            const int64_t sh = i * w - b0;
            acc |= sh >= 0 ? (code << sh) : (code >> (-sh));
        }
        it.dst[q] = (uint32_t)acc;
    }
}

// One item per blockIdx.y; element (i, j) of src goes to (j, i) of dst.
__global__ void transpose_kernel(const TransItem* items) {
    const TransItem it = items[blockIdx.y];
    const int64_t count = it.m * it.n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / it.m, i = e - j * it.m;      // src column j, row i
        it.dst[i * it.ld_dst + j] = it.src[j * it.ld_src + i];
    }
}

// dst rows [0, rows_dst) of n columns: src rows [0, m), zeros below.
__global__ void copy2d_kernel(const CopyItem* items) {
    const CopyItem it = items[blockIdx.y];
    const int64_t count = it.rows_dst * it.n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = e / it.rows_dst, i = e - j * it.rows_dst;
        it.dst[j * it.ld_dst + i] = i < it.m ? it.src[j * it.ld_src + i] : 0.0;
    }
}

// ------------------------------------------------------------ launchers

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

void launch_qr_extract(const QrItem* items, int nitems, int64_t rows, int s, hipStream_t st) {
    dim3 grid(grid_for(rows * s, 1024), nitems);
    hipLaunchKernelGGL(qr_extract_kernel, grid, dim3(256), 0, st, items, rows, s);
}

void launch_qr_tinv(const QrItem* items, int nitems, int s, hipStream_t st) {
    dim3 grid(grid_for((int64_t)s * s, 64), nitems);
    hipLaunchKernelGGL(qr_tinv_kernel, grid, dim3(256), 0, st, items, s);
}

void launch_jacobi(const JacItem* items, int nitems, int s, hipStream_t st) {
    hipLaunchKernelGGL(jacobi_kernel, dim3(nitems), dim3(256), 0, st, items, s);
}

void launch_svd_to_jac(const JacItem* items, const double* U, const double* Vt, int nitems, int s,
                       hipStream_t st) {
    dim3 grid(grid_for((int64_t)s * s, 64), nitems);
    hipLaunchKernelGGL(svd_to_jac_kernel, grid, dim3(256), 0, st, items, U, Vt, s);
}

void launch_maxabs(const SumItem* items, int nitems, double* out, hipStream_t s) {
    hipLaunchKernelGGL(maxabs_kernel, dim3(nitems), dim3(256), 0, s, items, out);
}

void launch_transpose(const TransItem* items, int nitems, int64_t max_count, hipStream_t s) {
    dim3 grid(grid_for(max_count, 4096), nitems);
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, items);
}

void launch_copy2d(const CopyItem* items, int nitems, int64_t max_count, hipStream_t s) {
    dim3 grid(grid_for(max_count, 4096), nitems);
    hipLaunchKernelGGL(copy2d_kernel, grid, dim3(256), 0, s, items);
}

void launch_pack_cont(const ContPackItem* items, int nitems, int64_t max_dwords, hipStream_t s) {
    dim3 grid(grid_for(max_dwords, 2048), nitems);
    hipLaunchKernelGGL(pack_cont_kernel, grid, dim3(256), 0, s, items);
}

void launch_pack(const PackItem* items, int nitems, int64_t max_count, hipStream_t s) {
    dim3 grid(grid_for(max_count, 2048), nitems);
    hipLaunchKernelGGL(pack_kernel, grid, dim3(256), 0, s, items);
}

}  // namespace hh
