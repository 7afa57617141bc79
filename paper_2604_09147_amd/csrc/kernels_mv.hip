// Product kernels of Alg. 4 on gfx950: b = sum_b U_b (V_b^T x_J) + sum D x.
//
// Phase 1 (gather):  xt = x in padded tree order (fp64).
// Phase 2 (dot):     one coefficient per stored column, tb[c] = V_c . xt_J
//                    (for the transpose, U_c . xt_I). One workgroup per task of
//                    columns; a wave owns a column, each lane 4 consecutive rows.
// Phase 3 (axpy):    one workgroup per leaf owns that leaf's output rows and
//                    accumulates every column segment covering them
//                    (U_c[leaf rows] tb[c] scale_b), the dense blocks, and, for
//                    the transpose, the in-kernel transposed dense blocks; then
//                    writes y in caller order. No atomics: results are bitwise
//                    reproducible.
// Factors stored in fp32 / fp64 and dense blocks use fp64 arithmetic; fp16 and
// bf16 columns multiply and accumulate their lane partials in fp32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hh_internal.h"

namespace hh {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

__device__ inline float bf16lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ inline float bf16hi(uint32_t u) { return __uint_as_float(u & 0xFFFF0000u); }

// Four consecutive elements starting at element index i (i multiple of 4).
template <int FMT>
__device__ inline void ld4(const void* base, int64_t i, double v[4]) {
    if constexpr (FMT == HH_FMT_FP64) {
        const double2* p = reinterpret_cast<const double2*>(static_cast<const double*>(base) + i);
        double2 a = p[0], b = p[1];
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    } else if constexpr (FMT == HH_FMT_FP32) {
        float4 f = *reinterpret_cast<const float4*>(static_cast<const float*>(base) + i);
        v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
    } else if constexpr (FMT == HH_FMT_FP16) {
        half4_t h = *reinterpret_cast<const half4_t*>(static_cast<const _Float16*>(base) + i);
        v[0] = (float)h.x; v[1] = (float)h.y; v[2] = (float)h.z; v[3] = (float)h.w;
    } else {
        uint2 u = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(base) + i);
        v[0] = bf16lo(u.x); v[1] = bf16hi(u.x); v[2] = bf16lo(u.y); v[3] = bf16hi(u.y);
    }
}

template <int FMT>
__device__ inline void ld4f(const void* base, int64_t i, float v[4]) {
    if constexpr (FMT == HH_FMT_FP16) {
        half4_t h = *reinterpret_cast<const half4_t*>(static_cast<const _Float16*>(base) + i);
        v[0] = (float)h.x; v[1] = (float)h.y; v[2] = (float)h.z; v[3] = (float)h.w;
    } else {
        uint2 u = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(base) + i);
        v[0] = bf16lo(u.x); v[1] = bf16hi(u.x); v[2] = bf16lo(u.y); v[3] = bf16hi(u.y);
    }
}

template <int FMT>
__device__ inline const void* col_ptr(const void* base, int64_t elems) {
    if constexpr (FMT == HH_FMT_FP64) return static_cast<const double*>(base) + elems;
    else if constexpr (FMT == HH_FMT_FP32) return static_cast<const float*>(base) + elems;
    else return static_cast<const uint16_t*>(base) + elems;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------------ gather
__global__ void gather_kernel(Desc d, const Desc* descs, int R) {
    const Desc D = descs ? descs[blockIdx.y] : d;
    const int64_t total = D.np * R;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t p = idx / R, r = idx - p * R;
        int64_t u = D.pmap[p];
        double v = 0.0;
        if (u >= 0) {
            if (D.io == HH_IO_F64) v = static_cast<const double*>(D.x)[u * R + r];
            else v = (double)static_cast<const float*>(D.x)[u * R + r];
        }
        D.xt[idx] = v;
    }
}

// --------------------------------------------------------------------- dot
constexpr int XLDS = 4096;   // rows of xt staged in LDS for single-vector tasks

template <int FMT>
__device__ void dot_task_r1(const DotTask& t, const double* x, const double* xs, bool lds,
                            double* tb, int wave, int lane) {
    const int P = t.P;
    for (int c = wave; c < t.ncols; c += 4) {
        const void* col = col_ptr<FMT>(t.col0, (int64_t)c * P);
        double acc;
        if constexpr (FMT >= HH_FMT_FP16) {
            float a0 = 0.f, a1 = 0.f;
            int r = 4 * lane;
            for (; r + 256 < P; r += 512) {
                float v[4], w[4];
                ld4f<FMT>(col, r, v);
                ld4f<FMT>(col, r + 256, w);
                const double* xa = lds ? xs + r : x + r;
                const double* xb = lds ? xs + r + 256 : x + r + 256;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a0 = fmaf(v[q], (float)xa[q], a0);
                    a1 = fmaf(w[q], (float)xb[q], a1);
                }
            }
            if (r < P) {
                float v[4];
                ld4f<FMT>(col, r, v);
                const double* xa = lds ? xs + r : x + r;
#pragma unroll
                for (int q = 0; q < 4; ++q) a0 = fmaf(v[q], (float)xa[q], a0);
            }
            acc = (double)a0 + (double)a1;
        } else {
            double a0 = 0.0, a1 = 0.0;
            int r = 4 * lane;
            for (; r + 256 < P; r += 512) {
                double v[4], w[4];
                ld4<FMT>(col, r, v);
                ld4<FMT>(col, r + 256, w);
                const double* xa = lds ? xs + r : x + r;
                const double* xb = lds ? xs + r + 256 : x + r + 256;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a0 = fma(v[q], xa[q], a0);
                    a1 = fma(w[q], xb[q], a1);
                }
            }
            if (r < P) {
                double v[4];
                ld4<FMT>(col, r, v);
                const double* xa = lds ? xs + r : x + r;
#pragma unroll
                for (int q = 0; q < 4; ++q) a0 = fma(v[q], xa[q], a0);
            }
            acc = a0 + a1;
        }
        acc = wave_sum(acc);
        if (lane == 0) tb[t.toff + c] = acc;
    }
}

// Several right-hand sides, RC at a time (columns re-read per chunk).
template <int FMT, int RC>
__device__ void dot_task_rn(const DotTask& t, const double* xt, double* tb, int R, int wave,
                            int lane) {
    const int P = t.P;
    for (int r0 = 0; r0 < R; r0 += RC) {
        const int nr = R - r0 < RC ? R - r0 : RC;
        for (int c = wave; c < t.ncols; c += 4) {
            const void* col = col_ptr<FMT>(t.col0, (int64_t)c * P);
            double acc[RC];
#pragma unroll
            for (int k = 0; k < RC; ++k) acc[k] = 0.0;
            if constexpr (FMT >= HH_FMT_FP16) {
                float fa[RC];
#pragma unroll
                for (int k = 0; k < RC; ++k) fa[k] = 0.f;
                for (int r = 4 * lane; r < P; r += 256) {
                    float v[4];
                    ld4f<FMT>(col, r, v);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double* xr = xt + (t.xoff + r + q) * R + r0;
#pragma unroll
                        for (int k = 0; k < RC; ++k)
                            if (k < nr) fa[k] = fmaf(v[q], (float)xr[k], fa[k]);
                    }
                }
#pragma unroll
                for (int k = 0; k < RC; ++k) acc[k] = fa[k];
            } else {
                for (int r = 4 * lane; r < P; r += 256) {
                    double v[4];
                    ld4<FMT>(col, r, v);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double* xr = xt + (t.xoff + r + q) * R + r0;
#pragma unroll
                        for (int k = 0; k < RC; ++k)
                            if (k < nr) acc[k] = fma(v[q], xr[k], acc[k]);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < RC; ++k) {
                double s = wave_sum(acc[k]);
                if (lane == 0 && k < nr) tb[(t.toff + c) * R + r0 + k] = s;
            }
        }
    }
}

__global__ __launch_bounds__(256) void dot_kernel(Desc d, const Desc* descs,
                                                  const DotTask* tasks, int R) {
    __shared__ double xs[XLDS];
    const DotTask t = tasks[blockIdx.x];
    const Desc D = descs ? descs[t.hid] : d;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (R == 1) {
        const double* x = D.xt + t.xoff;
        const bool lds = t.P <= XLDS;
        if (lds) {
            for (int i = tid; i < t.P; i += 256) xs[i] = x[i];
            __syncthreads();
        }
        switch (t.fmt) {
            case HH_FMT_FP64: dot_task_r1<HH_FMT_FP64>(t, x, xs, lds, D.tb, wave, lane); break;
            case HH_FMT_FP32: dot_task_r1<HH_FMT_FP32>(t, x, xs, lds, D.tb, wave, lane); break;
            case HH_FMT_FP16: dot_task_r1<HH_FMT_FP16>(t, x, xs, lds, D.tb, wave, lane); break;
            default: dot_task_r1<HH_FMT_BF16>(t, x, xs, lds, D.tb, wave, lane); break;
        }
    } else {
        switch (t.fmt) {
            case HH_FMT_FP64: dot_task_rn<HH_FMT_FP64, 8>(t, D.xt, D.tb, R, wave, lane); break;
            case HH_FMT_FP32: dot_task_rn<HH_FMT_FP32, 8>(t, D.xt, D.tb, R, wave, lane); break;
            case HH_FMT_FP16: dot_task_rn<HH_FMT_FP16, 8>(t, D.xt, D.tb, R, wave, lane); break;
            default: dot_task_rn<HH_FMT_BF16, 8>(t, D.xt, D.tb, R, wave, lane); break;
        }
    }
}

// -------------------------------------------------------------------- axpy
template <int FMT, int RC>
__device__ inline void axpy_run(const Run& rn, const double* coef, int R, int r0, int nr,
                                int gg, int TG, int64_t row, bool active, double acc[4][RC]) {
    for (int c = gg; c < rn.ncols; c += TG) {
        double cf[RC];
        const double* cp = coef + (rn.toff + c) * R + r0;
#pragma unroll
        for (int k = 0; k < RC; ++k) cf[k] = k < nr ? cp[k] * rn.scale : 0.0;
        if (active) {
            double v[4];
            ld4<FMT>(rn.base, (int64_t)c * rn.stride + row, v);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int k = 0; k < RC; ++k) acc[q][k] = fma(v[q], cf[k], acc[q][k]);
        }
    }
}

template <int RC>
__device__ void axpy_leaf(const Desc& D, const LeafTask& L, const Run* runs, const DotRun* druns,
                          int R) {
    __shared__ double part[256 * RC];
    __shared__ double ydot[256 * RC];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int P = L.P;
    int lps = 1;
    while (lps < 64 && 4 * lps < P) lps <<= 1;      // lanes per column segment
    const int G = 64 / lps;                          // segments per wave
    const int TG = 4 * G;                            // segments per workgroup
    const int g = lane / lps, sl = lane % lps, gg = wave * G + g;
    const int rows_per_stripe = 4 * lps;
    const int nstripes = (P + rows_per_stripe - 1) / rows_per_stripe;

    for (int r0 = 0; r0 < R; r0 += RC) {
        const int nr = R - r0 < RC ? R - r0 : RC;
        for (int s = 0; s < nstripes; ++s) {
            const int64_t row = (int64_t)4 * (sl + (int64_t)lps * s);
            const bool active = row < P;
            double acc[4][RC];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int k = 0; k < RC; ++k) acc[q][k] = 0.0;
            for (int ri = L.run_begin; ri < L.run_end; ++ri) {
                const Run rn = runs[ri];
                const double* coef = rn.from_x ? D.xt : D.tb;
                switch (rn.fmt) {
                    case HH_FMT_FP64: axpy_run<HH_FMT_FP64, RC>(rn, coef, R, r0, nr, gg, TG, row, active, acc); break;
                    case HH_FMT_FP32: axpy_run<HH_FMT_FP32, RC>(rn, coef, R, r0, nr, gg, TG, row, active, acc); break;
                    case HH_FMT_FP16: axpy_run<HH_FMT_FP16, RC>(rn, coef, R, r0, nr, gg, TG, row, active, acc); break;
                    default: axpy_run<HH_FMT_BF16, RC>(rn, coef, R, r0, nr, gg, TG, row, active, acc); break;
                }
            }
            // combine the segments of one wave that cover the same rows
            for (int off = lps; off < 64; off <<= 1)
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int k = 0; k < RC; ++k) acc[q][k] += __shfl_xor(acc[q][k], off, 64);
            // combine the waves in a fixed order
            for (int w = 0; w < 4; ++w) {
                if (wave == w && g == 0)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int k = 0; k < RC; ++k) {
                            double& dst = part[(4 * sl + q) * RC + k];
                            dst = (w == 0 ? 0.0 : dst) + acc[q][k];
                        }
                __syncthreads();
            }
            // transposed dense blocks: y_mu[j] += dot(D[:, j], xt_lambda)
            for (int i = tid; i < rows_per_stripe * RC; i += 256) ydot[i] = 0.0;
            __syncthreads();
            const int jlo = s * rows_per_stripe;
            for (int di = L.drun_begin; di < L.drun_end; ++di) {
                const DotRun dr = druns[di];
                const int jhi = dr.ncols < jlo + rows_per_stripe ? dr.ncols : jlo + rows_per_stripe;
                for (int j = jlo + wave; j < jhi; j += 4) {
                    const double* col = dr.base + (int64_t)j * dr.P;
                    double a[RC];
#pragma unroll
                    for (int k = 0; k < RC; ++k) a[k] = 0.0;
                    for (int i = lane; i < dr.P; i += 64) {
                        const double v = col[i];
                        const double* xr = D.xt + (dr.xoff + i) * R + r0;
#pragma unroll
                        for (int k = 0; k < RC; ++k)
                            if (k < nr) a[k] = fma(v, xr[k], a[k]);
                    }
#pragma unroll
                    for (int k = 0; k < RC; ++k) {
                        double t = wave_sum(a[k]);
                        if (lane == 0) ydot[(j - jlo) * RC + k] += t;
                    }
                }
            }
            __syncthreads();
            // write this stripe of y in caller order
            for (int i = tid; i < rows_per_stripe * RC; i += 256) {
                const int rr = i / RC, k = i - rr * RC;
                const int64_t prow = (int64_t)jlo + rr;
                if (prow < P && k < nr) {
                    const int64_t u = D.pmap[L.poff + prow];
                    if (u >= 0) {
                        const double v = part[rr * RC + k] + ydot[rr * RC + k];
                        if (D.io == HH_IO_F64) static_cast<double*>(D.y)[u * R + r0 + k] = v;
                        else static_cast<float*>(D.y)[u * R + r0 + k] = (float)v;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(256) void axpy_kernel(Desc d, const Desc* descs,
                                                   const LeafTask* leaves, const Run* runs,
                                                   const DotRun* druns, int R) {
    const LeafTask L = leaves[blockIdx.x];
    const Desc D = descs ? descs[L.hid] : d;
    if (R == 1) axpy_leaf<1>(D, L, runs, druns, R);
    else axpy_leaf<4>(D, L, runs, druns, R);
}

// ------------------------------------------------------------- launchers
void launch_gather(const Desc& d, const Desc* descs, int nh, int64_t max_np, int R, void* stream) {
    int64_t total = max_np * R;
    int64_t g = (total + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)g, nh), dim3(256), 0, (hipStream_t)stream, d,
                       descs, R);
}

void launch_dot(const Desc& d, const Desc* descs, const DotTask* tasks, int64_t ntasks, int R,
                void* stream) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(dot_kernel, dim3((unsigned)ntasks), dim3(256), 0, (hipStream_t)stream, d,
                       descs, tasks, R);
}

void launch_axpy(const Desc& d, const Desc* descs, const LeafTask* leaves, int64_t nleaves,
                 const Run* runs, const DotRun* druns, int R, void* stream) {
    if (nleaves <= 0) return;
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)nleaves), dim3(256), 0, (hipStream_t)stream, d,
                       descs, leaves, runs, druns, R);
}

}  // namespace hh
