// Product kernels of Alg. 4 on gfx950: b = sum_b U_b (V_b^T x_J) + sum D x.
//
// Phase 1 (gather):     xt = x in padded tree order (fp64).
// Phase 2 (dot):        one coefficient per stored column, tb[c] = 2^e V_c . xt_J
//                       (for the transpose, U_c . xt_I), e the block's factor
//                       scales. One workgroup per task of columns of one block;
//                       every wave keeps eight independent 16-byte loads per lane
//                       in flight (several columns of a short column length, or
//                       several 256-row pieces of a long one).
// Phase 3 (accumulate): the output rows of a leaf box are the sum, over the
//                       clusters that contain the leaf (one per level), of runs:
//                       strided column sets (the factors of the cluster's blocks
//                       of one storage format, or a dense block) times their
//                       coefficients tb (low-rank) or xt (dense). One RHS: each
//                       leaf's runs are cut into work units of about 1 MB, one
//                       wave each, writing partial rows that a finishing kernel
//                       adds in unit order and writes to y in caller order.
//                       Several RHS: fp64 MFMA on 16-column tiles (phase V) and
//                       on 64-row leaf slices over the cluster runs (phase U).
//                       Run records and coefficients are wave-uniform (scalar
//                       loads); factor data goes through buffer loads. No atomics
//                       and a fixed order: results are bitwise reproducible.
// Factors stored in fp32 / fp64 and dense blocks use fp64 arithmetic; fp16 and
// bf16 inner products multiply and accumulate their lane partials in fp32.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hh_internal.h"

namespace hh {

// Native vector types (HIP's double2 / float4 wrappers copy through a generic
// pointer and would turn every load below back into a flat access).
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef double dbl2_t __attribute__((ext_vector_type(2)));
typedef float flt4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

// Loads through the global address space (vector memory path) and through the
// constant address space (scalar loads when the address is wave-uniform).
// Pointers read out of task records are generic; without these casts every
// access would be a flat access, which also holds the LDS / scalar counter.
template <class T>
__device__ inline T ldg(const void* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ inline T ldc(const void* p) {
    return *(const __attribute__((address_space(4))) T*)p;
}
// A task record read as 64-bit words through the constant address space, so
// that a wave-uniform record lands in scalar registers (an aggregate copy
// would go through a generic pointer).
template <class T>
__device__ inline T ldrec(const T* p) {
    static_assert(sizeof(T) % 8 == 0, "records are whole 64-bit words");
    uint64_t w[sizeof(T) / 8];
#pragma unroll
    for (size_t i = 0; i < sizeof(T) / 8; ++i) w[i] = ldc<uint64_t>(reinterpret_cast<const uint64_t*>(p) + i);
    T r;
    __builtin_memcpy(&r, w, sizeof(T));
    return r;
}
template <class T>
__device__ inline void stg(void* p, T v) {
    *(__attribute__((address_space(1))) T*)p = v;
}

// Four consecutive stored elements, still in their storage format.
template <int FMT> struct Raw4;
template <> struct Raw4<HH_FMT_FP64> { dbl2_t a, b; };
template <> struct Raw4<HH_FMT_FP32> { flt4_t a; };
template <> struct Raw4<HH_FMT_FP16> { half4_t a; };
template <> struct Raw4<HH_FMT_BF16> { u32x2_t a; };
template <> struct Raw4<HH_FMT_Q43> { uint32_t a; };

template <int FMT>
__device__ inline const void* elem_ptr(const void* base, int64_t i) {
    if constexpr (FMT == HH_FMT_FP64) return static_cast<const double*>(base) + i;
    else if constexpr (FMT == HH_FMT_FP32) return static_cast<const float*>(base) + i;
    else if constexpr (FMT == HH_FMT_Q43) return static_cast<const uint8_t*>(base) + i;
    else return static_cast<const uint16_t*>(base) + i;
}

// A global load marked non-temporal: factor data is read once per product, so
// it should not displace the vectors and coefficients held in the caches.
template <class T>
__device__ inline T ldg_nt(const void* p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}

// Elements i .. i+3 (i a multiple of 4, so the access is aligned); NT: a
// non-temporal load.
template <int FMT, bool NT = false>
__device__ inline Raw4<FMT> load4(const void* base, int64_t i) {
    Raw4<FMT> r;
    const void* p = elem_ptr<FMT>(base, i);
    if constexpr (FMT == HH_FMT_FP64) {
        // two loads share each cache line: no streaming hint (see bload4)
        r.a = ldg<dbl2_t>(p);
        r.b = ldg<dbl2_t>(static_cast<const dbl2_t*>(p) + 1);
    } else if constexpr (FMT == HH_FMT_FP32) {
        r.a = NT ? ldg_nt<flt4_t>(p) : ldg<flt4_t>(p);
    } else if constexpr (FMT == HH_FMT_FP16) {
        r.a = NT ? ldg_nt<half4_t>(p) : ldg<half4_t>(p);
    } else if constexpr (FMT == HH_FMT_Q43) {
        r.a = NT ? ldg_nt<uint32_t>(p) : ldg<uint32_t>(p);
    } else {
        r.a = NT ? ldg_nt<u32x2_t>(p) : ldg<u32x2_t>(p);
    }
    return r;
}

// Buffer loads: a resource descriptor (base, byte size) in scalar registers
// and a 32-bit byte offset per lane, so an address costs one vector register.
// An offset at or past the descriptor's size reads zero instead of faulting.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;   // raw 32-bit data format (gfx9 family)

__device__ inline rsrc_t make_rsrc(const void* base, int64_t bytes) {
    const int nrec = bytes < 0x7fffffff ? (int)bytes : 0x7fffffff;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nrec, RSRC_WORD3);
}

// Cache policy of a buffer load: CP_STREAM marks it non-temporal (the
// single-vector kernels read every factor byte once per product; measured at
// the benchmark size, the product is 6% faster with it). fp64 factors are
// loaded as two 16-byte halves per lane and keep the default policy, and so do
// the several-RHS kernels, whose right-hand-side groups re-read a tile's
// columns from L2.
constexpr int CP_STREAM = 2;

// Elements at byte offset off .. off + 4 elements of a buffer.
template <int FMT, int CP = 0>
__device__ inline Raw4<FMT> bload4(rsrc_t rs, uint32_t off) {
    Raw4<FMT> r;
    if constexpr (FMT == HH_FMT_FP64) {
        // two loads share each cache line: no streaming hint, or the line can
        // leave the cache between them
        r.a = __builtin_bit_cast(dbl2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
        r.b = __builtin_bit_cast(dbl2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0));
    } else if constexpr (FMT == HH_FMT_FP32) {
        r.a = __builtin_bit_cast(flt4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, CP));
    } else if constexpr (FMT == HH_FMT_FP16) {
        r.a = __builtin_bit_cast(half4_t, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, CP));
    } else if constexpr (FMT == HH_FMT_Q43) {
        r.a = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, CP);
    } else {
        r.a = __builtin_bit_cast(u32x2_t, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, CP));
    }
    return r;
}

template <int FMT>
constexpr int elem_bytes() {
    return FMT == HH_FMT_FP64 ? 8 : FMT == HH_FMT_FP32 ? 4 : FMT == HH_FMT_Q43 ? 1 : 2;
}

// Two q43 codes, at bits 8..15 and 24..31 of t, as two fp16 (low, high half):
// sign to bit 15, exponent field and fraction to bits 7..14, which is the
// code's value times 2^-8 (exact, subnormals included).
__device__ inline uint32_t q43_pair_to_h16(uint32_t t) {
    return ((t >> 1) & 0x3F803F80u) | (t & 0x80008000u);
}

__device__ inline float bf16lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ inline float bf16hi(uint32_t u) { return __uint_as_float(u & 0xFFFF0000u); }

// Exact widening to T (float for the 16- and 8-bit formats, double otherwise).
template <int FMT, typename T>
__device__ inline void widen4(const Raw4<FMT>& r, T v[4]) {
    if constexpr (FMT == HH_FMT_FP64) {
        v[0] = r.a.x; v[1] = r.a.y; v[2] = r.b.x; v[3] = r.b.y;
    } else if constexpr (FMT == HH_FMT_FP32) {
        v[0] = r.a.x; v[1] = r.a.y; v[2] = r.a.z; v[3] = r.a.w;
    } else if constexpr (FMT == HH_FMT_FP16) {
        v[0] = (float)r.a.x; v[1] = (float)r.a.y; v[2] = (float)r.a.z; v[3] = (float)r.a.w;
    } else if constexpr (FMT == HH_FMT_Q43) {
        // 2^-8 times the stored values (the block's coefficient carries 2^16)
        const uint32_t lo = q43_pair_to_h16(((r.a << 8) & 0x0000FF00u) | ((r.a << 16) & 0xFF000000u));
        const uint32_t hi = q43_pair_to_h16(((r.a >> 8) & 0x0000FF00u) | (r.a & 0xFF000000u));
        const half4_t h = __builtin_bit_cast(half4_t, u32x2_t{lo, hi});
        v[0] = (float)h.x; v[1] = (float)h.y; v[2] = (float)h.z; v[3] = (float)h.w;
    } else {
        v[0] = bf16lo(r.a.x); v[1] = bf16hi(r.a.x); v[2] = bf16lo(r.a.y); v[3] = bf16hi(r.a.y);
    }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }


// ------------------------------------------------------ continuum storage
// A continuum column holds its entries back to back, W = 9 + t bits each, in
// little-endian bit order (entry i at bits [i W, i W + W) of the column); an
// entry is the top W bits of the fp32 encoding of its value. Columns start at
// 16-byte boundaries (cont_col_bytes). A lane owning 4 consecutive entries
// loads the 4 dwords that hold them (5 when W > 24) from the dword holding
// the first one, shifts the words down by the first entry's bit offset in that
// dword (a per-lane funnel shift), after which entry j sits at bit j W for
// every lane: extracting it is one more funnel shift by a compile-time amount
// and a left shift that drops the next entry's bits. The values are exact fp32
// numbers, widened exactly to fp64.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Byte-aligned widths (16, 24 and 32 bits: t = 7, 15, 23) put a lane's four
// entries in whole dwords of their own (2, 3 or 4, at a lane stride of W / 2
// bytes), so they load without overlap and decode without the funnel shift:
// the 24-bit entries are byte permutes into the top three bytes of a word.
template <int W>
constexpr int craw_words() { return W == 16 ? 2 : W == 24 ? 3 : W == 32 ? 4 : W > 24 ? 5 : 4; }
template <int W>
struct CRaw { uint32_t d[craw_words<W>()]; };

// Byte offset of the dword holding entry `row` of a column, and the entry's
// bit offset inside it.
template <int W>
__device__ inline void cpos(int64_t row, uint32_t& off, uint32_t& sh) {
    const uint64_t bit = (uint64_t)row * W;
    off = (uint32_t)(bit >> 5) << 2;
    sh = (uint32_t)bit & 31u;
}

typedef uint32_t u32x3_t __attribute__((ext_vector_type(3)));

template <int W, int CP = 0>
__device__ inline CRaw<W> cload(rsrc_t rs, uint32_t off) {
    CRaw<W> r;
    if constexpr (W == 16) {
        const u32x2_t v = __builtin_bit_cast(u32x2_t, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, CP));
        r.d[0] = v.x; r.d[1] = v.y;
    } else if constexpr (W == 24) {
        const u32x3_t v = __builtin_bit_cast(u32x3_t, __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, CP));
        r.d[0] = v.x; r.d[1] = v.y; r.d[2] = v.z;
    } else {
        const u32x4_t v = __builtin_bit_cast(u32x4_t, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, CP));
        r.d[0] = v.x; r.d[1] = v.y; r.d[2] = v.z; r.d[3] = v.w;
        if constexpr (W > 24 && W < 32) r.d[4] = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 16, 0, CP);
    }
    return r;
}

template <int W>
__device__ inline void cwiden(const CRaw<W>& r, uint32_t sh, double v[4]) {
    if constexpr (W == 16) {
        v[0] = (double)__uint_as_float(r.d[0] << 16);
        v[1] = (double)__uint_as_float(r.d[0] & 0xFFFF0000u);
        v[2] = (double)__uint_as_float(r.d[1] << 16);
        v[3] = (double)__uint_as_float(r.d[1] & 0xFFFF0000u);
        return;
    } else if constexpr (W == 24) {
        // entry j = bits [24 j, 24 j + 24); byte 0 of every result is zero
        v[0] = (double)__uint_as_float(__builtin_amdgcn_perm(r.d[1], r.d[0], 0x0201000Cu));
        v[1] = (double)__uint_as_float(__builtin_amdgcn_perm(r.d[1], r.d[0], 0x0504030Cu));
        v[2] = (double)__uint_as_float(__builtin_amdgcn_perm(r.d[2], r.d[1], 0x0403020Cu));
        v[3] = (double)__uint_as_float(r.d[2] & 0xFFFFFF00u);
        return;
    } else if constexpr (W == 32) {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (double)__uint_as_float(r.d[j]);
        return;
    }
    uint32_t e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t hi = 0u;
        if constexpr (W > 24) hi = r.d[k + 1 < craw_words<W>() ? k + 1 : k];
        else if (k < 3) hi = r.d[k + 1];
        e[k] = __builtin_amdgcn_alignbit(hi, r.d[k], sh);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int pos = j * W, k = pos >> 5, s = pos & 31;
        const uint32_t win = s == 0 ? e[k] : __builtin_amdgcn_alignbit(e[k + 1 < 4 ? k + 1 : 3], e[k], s);
        v[j] = (double)__uint_as_float(win << (32 - W));
    }
}

// Calls F.template operator()<W>() for the run-time width w (16..32).
template <class F>
__device__ inline void with_width(int w, F&& f) {
    switch (w) {
        case 16: f.template operator()<16>(); break;
        case 17: f.template operator()<17>(); break;
        case 18: f.template operator()<18>(); break;
        case 19: f.template operator()<19>(); break;
        case 20: f.template operator()<20>(); break;
        case 21: f.template operator()<21>(); break;
        case 22: f.template operator()<22>(); break;
        case 23: f.template operator()<23>(); break;
        case 24: f.template operator()<24>(); break;
        case 25: f.template operator()<25>(); break;
        case 26: f.template operator()<26>(); break;
        case 27: f.template operator()<27>(); break;
        case 28: f.template operator()<28>(); break;
        case 29: f.template operator()<29>(); break;
        case 30: f.template operator()<30>(); break;
        case 31: f.template operator()<31>(); break;
        default: f.template operator()<32>(); break;
    }
}

// ------------------------------------------------------------------ gather
__global__ void gather_kernel(Desc d, const Desc* descs, int R) {
    const Desc D = descs ? ldrec<Desc>(descs + blockIdx.y) : d;
    const int64_t total = D.np * R;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t p = idx / R, r = idx - p * R;
        const int64_t u = ldg<int64_t>(D.pmap + p);
        double v = 0.0;
        if (u >= 0) {
            if (D.io == HH_IO_F64) v = ldg<double>(static_cast<const double*>(D.x) + u * R + r);
            else v = (double)ldg<float>(static_cast<const float*>(D.x) + u * R + r);
        }
        stg<double>(D.xt + idx, v);
    }
}

// --------------------------------------------------------------------- dot

// One iteration of a wave covers UC columns x UR pieces of 256 rows (UC UR =
// NU, eight loads of 16 bytes per lane; four of 32 bytes for fp64).
// Units past the last column or row re-read an in-bounds element and are
// discarded (column clamped, weight zero), so every load is unconditional.
// PANEL: the task's columns may belong to several blocks (a panel task);
// column c's coefficient index and exponent come from t.cmap[c].
template <int FMT, int UR, int NU = 8, bool PANEL = false>
__device__ void dot_r1(const DotTask& t, const double* xg, const double* xs, bool lds,
                       double* tb, int wave, int lane) {
    constexpr int UC = (FMT == HH_FMT_FP64 ? NU / 2 : NU) / UR;
    using acc_t = typename std::conditional<(FMT >= HH_FMT_FP16), float, double>::type;
    const int P = t.P;
    for (int c0 = wave * UC; c0 < t.ncols; c0 += 4 * UC) {
        acc_t a[UC];
#pragma unroll
        for (int u = 0; u < UC; ++u) a[u] = 0;
        for (int rb = 0; rb < P; rb += 256 * UR) {
            Raw4<FMT> raw[UC][UR];
#pragma unroll
            for (int uc = 0; uc < UC; ++uc) {
                const int c = c0 + uc < t.ncols ? c0 + uc : t.ncols - 1;
#pragma unroll
                for (int ur = 0; ur < UR; ++ur) {
                    const int r = rb + 256 * ur + 4 * lane;
                    raw[uc][ur] = load4<FMT, true>(t.col0, (int64_t)c * P + (r < P ? r : 0));
                }
            }
#pragma unroll
            for (int ur = 0; ur < UR; ++ur) {
                const int r = rb + 256 * ur + 4 * lane;
                acc_t xv[4] = {0, 0, 0, 0};
                if (r < P) {
                    if (lds) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) xv[q] = (acc_t)xs[r + q];
                    } else {
                        const dbl2_t x0 = ldg<dbl2_t>(xg + r), x1 = ldg<dbl2_t>(xg + r + 2);
                        xv[0] = (acc_t)x0.x; xv[1] = (acc_t)x0.y; xv[2] = (acc_t)x1.x; xv[3] = (acc_t)x1.y;
                    }
                }
#pragma unroll
                for (int uc = 0; uc < UC; ++uc) {
                    acc_t v[4];
                    widen4<FMT, acc_t>(raw[uc][ur], v);
#pragma unroll
                    for (int q = 0; q < 4; ++q) a[uc] = fma(v[q], xv[q], a[uc]);
                }
            }
        }
#pragma unroll
        for (int uc = 0; uc < UC; ++uc) {
            if constexpr (PANEL) {
                const double s = wave_sum((double)a[uc]);
                if (lane == 0 && c0 + uc < t.ncols) {
                    const int64_t m = ldg<int64_t>(t.cmap + c0 + uc);
                    stg<double>(tb + (m & (((int64_t)1 << 40) - 1)), ldexp(s, (int)(m >> 40) - 1024));
                }
            } else {
                const double s = ldexp(wave_sum((double)a[uc]), t.exp);
                if (lane == 0 && c0 + uc < t.ncols) stg<double>(tb + t.toff + c0 + uc, s);
            }
        }
    }
}

template <int FMT, int NU, bool PANEL = false>
__device__ void dot_r1_any(const DotTask& t, const double* xg, const double* xs, bool lds,
                           double* tb, int wave, int lane) {
    constexpr int NF = FMT == HH_FMT_FP64 ? NU / 2 : NU;   // loads of 16 bytes per lane
    const int nb = (t.P + 255) / 256;
    constexpr int R2 = NF < 2 ? NF : 2, R4 = NF < 4 ? NF : 4, R8 = NF < 8 ? NF : 8;
    // x not staged in LDS (long columns): four columns per pass share each x
    // load (two for fp64)
    if (!lds && nb > 2) dot_r1<FMT, R2, NU, PANEL>(t, xg, xs, lds, tb, wave, lane);
    else if (nb <= 1) dot_r1<FMT, 1, NU, PANEL>(t, xg, xs, lds, tb, wave, lane);
    else if (nb <= 2) dot_r1<FMT, R2, NU, PANEL>(t, xg, xs, lds, tb, wave, lane);
    else if (nb <= 4) dot_r1<FMT, R4, NU, PANEL>(t, xg, xs, lds, tb, wave, lane);
    else dot_r1<FMT, R8, NU, PANEL>(t, xg, xs, lds, tb, wave, lane);
}

// Continuum columns: UC columns x UR pieces of 256 rows per wave iteration,
// fp64 accumulation, the per-lane bit position computed once per piece.
template <int W, int UR>
__device__ __forceinline__ void dot_cont(const DotTask& t, const double* xg, const double* xs,
                                         bool lds, double* tb, int wave, int lane) {
    constexpr int NL = W > 24 ? 4 : 8;             // loads in flight (5-dword loads above 24 bits)
    constexpr int UC = NL / UR > 0 ? NL / UR : 1;
    const int P = t.P;
    const uint32_t cb = (uint32_t)cont_col_bytes(P, W);
    const rsrc_t rs = make_rsrc(t.col0, (int64_t)t.ncols * cb);
    for (int c0 = wave * UC; c0 < t.ncols; c0 += 4 * UC) {
        double a[UC];
#pragma unroll
        for (int u = 0; u < UC; ++u) a[u] = 0.0;
        for (int rb = 0; rb < P; rb += 256 * UR) {
            CRaw<W> raw[UC][UR];
            uint32_t sh[UR];
#pragma unroll
            for (int ur = 0; ur < UR; ++ur) {
                const int r = rb + 256 * ur + 4 * lane;
                uint32_t off;
                cpos<W>(r < P ? r : 0, off, sh[ur]);
#pragma unroll
                for (int uc = 0; uc < UC; ++uc) {
                    const int c = c0 + uc < t.ncols ? c0 + uc : t.ncols - 1;
                    raw[uc][ur] = cload<W, CP_STREAM>(rs, off + (uint32_t)c * cb);
                }
            }
#pragma unroll
            for (int ur = 0; ur < UR; ++ur) {
                const int r = rb + 256 * ur + 4 * lane;
                double xv[4] = {0.0, 0.0, 0.0, 0.0};
                if (r < P) {
                    if (lds) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) xv[q] = xs[r + q];
                    } else {
                        const dbl2_t x0 = ldg<dbl2_t>(xg + r), x1 = ldg<dbl2_t>(xg + r + 2);
                        xv[0] = x0.x; xv[1] = x0.y; xv[2] = x1.x; xv[3] = x1.y;
                    }
                }
#pragma unroll
                for (int uc = 0; uc < UC; ++uc) {
                    double v[4];
                    cwiden<W>(raw[uc][ur], sh[ur], v);
#pragma unroll
                    for (int q = 0; q < 4; ++q) a[uc] = fma(v[q], xv[q], a[uc]);
                }
            }
        }
#pragma unroll
        for (int uc = 0; uc < UC; ++uc) {
            const double s = ldexp(wave_sum(a[uc]), t.exp);
            if (lane == 0 && c0 + uc < t.ncols) stg<double>(tb + t.toff + c0 + uc, s);
        }
    }
}

struct DotCont {
    DotTask t;
    const double* xg;
    const double* xs;
    bool lds;
    double* tb;
    int wave, lane;
    template <int W>
    __device__ __forceinline__ void operator()() const {
        const int nb = (t.P + 255) / 256;
        if (!lds && nb > 1) dot_cont<W, 2>(t, xg, xs, lds, tb, wave, lane);
        else if (nb <= 1) dot_cont<W, 1>(t, xg, xs, lds, tb, wave, lane);
        else if (nb <= 2) dot_cont<W, 2>(t, xg, xs, lds, tb, wave, lane);
        else dot_cont<W, 4>(t, xg, xs, lds, tb, wave, lane);
    }
};

// FAM (FAM_FIX, FAM_CONT, FAM_Q43): the storage family of the launch. Handles
// with continuum storage hold continuum or fp64 low-rank blocks (a launch never
// mixes them with the 32- and 16-bit formats); q43 comes with the fixed
// formats. Each variant keeps only its own formats, so none pays the others'
// registers. PANEL: panel tasks (fixed formats and q43 only).
template <int NU, int XL, int FAM, bool PANEL = false>
__device__ inline void dot1_body(Desc d, const Desc* descs, const DotTask* tasks) {
    __shared__ double xs[XL];
    const DotTask t = ldrec<DotTask>(tasks + blockIdx.x);
    const Desc D = descs ? ldrec<Desc>(descs + t.hid) : d;
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const double* x = D.xt + t.xoff;
    const bool lds = t.P <= XL;
    if (lds) {
        for (int i = threadIdx.x; i < t.P; i += 256) xs[i] = ldg<double>(x + i);
        __syncthreads();
    }
    if constexpr (FAM == FAM_CONT) {
        static_assert(!PANEL, "no panel tasks over continuum storage");
        if (t.fmt == HH_FMT_CONT) with_width(t.w, DotCont{t, x, xs, lds, D.tb, wave, lane});
        else dot_r1_any<HH_FMT_FP64, NU>(t, x, xs, lds, D.tb, wave, lane);
    } else {
        if constexpr (FAM == FAM_Q43) {
            if (t.fmt == HH_FMT_Q43) {
                dot_r1_any<HH_FMT_Q43, NU, PANEL>(t, x, xs, lds, D.tb, wave, lane);
                return;
            }
        }
        switch (t.fmt) {
            case HH_FMT_FP64: dot_r1_any<HH_FMT_FP64, NU, PANEL>(t, x, xs, lds, D.tb, wave, lane); break;
            case HH_FMT_FP32: dot_r1_any<HH_FMT_FP32, NU, PANEL>(t, x, xs, lds, D.tb, wave, lane); break;
            case HH_FMT_FP16: dot_r1_any<HH_FMT_FP16, NU, PANEL>(t, x, xs, lds, D.tb, wave, lane); break;
            default: dot_r1_any<HH_FMT_BF16, NU, PANEL>(t, x, xs, lds, D.tb, wave, lane); break;
        }
    }
}

#define HH_DOT1_KERNEL(NAME, NU, XL, W, FAM)                                                    \
    __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void NAME(         \
        Desc d, const Desc* descs, const DotTask* tasks) {                                      \
        dot1_body<NU, XL, FAM>(d, descs, tasks);                                                \
    }
HH_DOT1_KERNEL(dot1_kernel, 8, 4096, 4, FAM_FIX)
HH_DOT1_KERNEL(dot1c_kernel, 8, 4096, 4, FAM_CONT)
HH_DOT1_KERNEL(dot1q_kernel, 8, 4096, 4, FAM_Q43)

// Panel tasks: the columns of consecutive blocks that share the x slice, the
// format and the stride, one task per DOT_TASK_ELEMS-sized piece of the panel
// (used when the blocks' own tasks would be a few KB each).
#define HH_DOT1P_KERNEL(NAME, FAM)                                                              \
    __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void NAME(         \
        Desc d, const Desc* descs, const DotTask* tasks) {                                      \
        dot1_body<8, 4096, FAM, true>(d, descs, tasks);                                         \
    }
HH_DOT1P_KERNEL(dot1p_kernel, FAM_FIX)
HH_DOT1P_KERNEL(dot1pq_kernel, FAM_Q43)

// -------------------------------------------------------------- accumulate
// Apply one run to a lane's 4 rows: acc += 2^e sum_c col_c[rows] coef_c
// (the power-of-two scale is exact, so applying it to the run's sum rounds as
// applying it to every coefficient would). SPLIT: the wave is cut into G
// groups of lps lanes (short leaves) and group g takes columns g, g + G, ...;
// without SPLIT the column index and so the coefficient address are
// wave-uniform.
// UB columns c, c + step, ... of one run (columns past the last one, only
// when CLAMP, re-read the last column with weight zero).
template <int FMT, int RC, int UB, bool CLAMP, bool SPLIT>
__device__ inline void apply_cols(const Run& rn, rsrc_t rs, uint32_t voff, const double* coef,
                                  int R, int r0, int nr, int c, int step, double ra[4][RC]) {
    const int n = rn.ncols;
    Raw4<FMT> raw[UB];
    double cf[UB][RC];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int cu = c + u * step;
        const int cc = CLAMP ? (cu < n ? cu : n - 1) : cu;
        raw[u] = bload4<FMT, CP_STREAM>(rs, voff + (uint32_t)cc * (uint32_t)rn.stride * elem_bytes<FMT>());
        const double* cp = coef + ((int64_t)rn.toff + cc) * R + r0;
#pragma unroll
        for (int k = 0; k < RC; ++k) {
            const double* ck = cp + (k < nr ? k : 0);
            cf[u][k] = SPLIT ? ldg<double>(ck) : ldc<double>(ck);
        }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const bool ok = !CLAMP || c + u * step < n;
        double v[4];
        widen4<FMT, double>(raw[u], v);
#pragma unroll
        for (int k = 0; k < RC; ++k) {
            const double w = (ok && k < nr) ? cf[u][k] : 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) ra[q][k] = fma(v[q], w, ra[q][k]);
        }
    }
}

// Apply one run to a lane's 4 rows: acc += sum_c col_c[rows] coef_c. Columns
// go in batches of U, then
// U/2 and U/4, and a clamped batch for the last few, so that short runs do
// not issue loads of absent columns. SPLIT: the wave is cut into G groups of
// lps lanes (short leaves) and group g takes columns g, g + G, ...; without
// SPLIT the column index and so the coefficient address are wave-uniform.
template <int FMT, int RC, bool SPLIT, int UB = 16>
__device__ inline void apply_run(const Run& rn, rsrc_t rs, uint32_t voff, const double* coef,
                                 int R, int r0, int nr, int g, int G, double acc[4][RC]) {
    constexpr int U = RC > 1 ? 2 : SPLIT ? 4 : FMT == HH_FMT_FP64 ? (UB < 8 ? UB : 8) : UB;
    const int n = rn.ncols;
    const int step = SPLIT ? G : 1;
    int c = SPLIT ? g : 0;
    for (; c + (U - 1) * step < n; c += U * step)
        apply_cols<FMT, RC, U, false, SPLIT>(rn, rs, voff, coef, R, r0, nr, c, step, acc);
    if constexpr (U >= 8) {
        if (c + (U / 2 - 1) * step < n) {
            apply_cols<FMT, RC, U / 2, false, SPLIT>(rn, rs, voff, coef, R, r0, nr, c, step, acc);
            c += (U / 2) * step;
        }
    }
    if constexpr (U >= 16) {
        if (c + (U / 4 - 1) * step < n) {
            apply_cols<FMT, RC, U / 4, false, SPLIT>(rn, rs, voff, coef, R, r0, nr, c, step, acc);
            c += (U / 4) * step;
        }
    }
    constexpr int T = U >= 16 ? U / 4 : U >= 8 ? U / 2 : U;
    if (c < n) apply_cols<FMT, RC, T, true, SPLIT>(rn, rs, voff, coef, R, r0, nr, c, step, acc);
}

// One run with software pipelining: the loads of batch b + 1 (UP columns) are
// issued before batch b is consumed, so a wave always has UP to 2 UP loads in
// flight; the last columns go through the tiered batches above.
template <int FMT, int UP>
__device__ inline void apply_run_pipe(const Run& rn, rsrc_t rs, uint32_t voff, const double* coef,
                                      double acc[4][1]) {
    const int n = rn.ncols;
    const int nb = n / UP;
    const uint32_t cstep = (uint32_t)rn.stride * elem_bytes<FMT>();
    if (nb > 0) {
        Raw4<FMT> cur[UP];
        double cfc[UP];
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            cur[u] = bload4<FMT, CP_STREAM>(rs, voff + (uint32_t)u * cstep);
            cfc[u] = ldc<double>(coef + rn.toff + u);
        }
        for (int b = 1; b < nb; ++b) {
            Raw4<FMT> nxt[UP];
            double cfn[UP];
#pragma unroll
            for (int u = 0; u < UP; ++u) {
                const int c = b * UP + u;
                nxt[u] = bload4<FMT, CP_STREAM>(rs, voff + (uint32_t)c * cstep);
                cfn[u] = ldc<double>(coef + rn.toff + c);
            }
#pragma unroll
            for (int u = 0; u < UP; ++u) {
                double v[4];
                widen4<FMT, double>(cur[u], v);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q][0] = fma(v[q], cfc[u], acc[q][0]);
            }
#pragma unroll
            for (int u = 0; u < UP; ++u) {
                cur[u] = nxt[u];
                cfc[u] = cfn[u];
            }
        }
#pragma unroll
        for (int u = 0; u < UP; ++u) {
            double v[4];
            widen4<FMT, double>(cur[u], v);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q][0] = fma(v[q], cfc[u], acc[q][0]);
        }
    }
    int c = nb * UP;
    if constexpr (UP >= 8) {
        if (c + UP / 2 - 1 < n) {
            apply_cols<FMT, 1, UP / 2, false, false>(rn, rs, voff, coef, 1, 0, 1, c, 1, acc);
            c += UP / 2;
        }
    }
    if (c < n) apply_cols<FMT, 1, 4, true, false>(rn, rs, voff, coef, 1, 0, 1, c, 1, acc);
}

// Index of the cluster of level l that contains leaf box `leaf`: clusters are
// numbered level by level, level l starting at sum_{l' < l} 2^(d l').
__device__ inline int64_t cluster_index(const Desc& D, int l, int64_t leaf) {
    int64_t first = 0;
    for (int i = 0; i < l; ++i) first += (int64_t)1 << (D.d * i);
    return first + (leaf >> (D.d * (D.L - l)));
}

// ---------------------------------------------- single-vector work units
// A unit is a slice of one leaf's runs (a few hundred KB to about 1 MB of
// factor data), so that the hardware dispatcher balances leaves of unequal
// work. Each unit writes its partial sum of the leaf's rows; the finishing
// kernel adds a leaf's partials in unit order.
template <int F, bool SPLIT, int UB>
__device__ inline void unit_runs_fmt(const Desc& D, const UnitTask& ut, int b, int e, int64_t row,
                                     int g, int G, double acc[4][1], bool pipe) {
    constexpr uint32_t es = elem_bytes<F>();
    if (b >= e) return;
    Run rn = ldrec<Run>(D.uruns + b);
    for (int i = b; i < e; ++i) {
        // the next record is requested before this run's factor loads
        const Run nx = ldrec<Run>(D.uruns + (i + 1 < e ? i + 1 : i));
        const double* coef = rn.from_x ? D.xt : D.tb;
        const int64_t off = ut.poff - rn.pc;
        const rsrc_t rs = make_rsrc(static_cast<const char*>(rn.base) + off * es,
                                    ((int64_t)rn.ncols * rn.stride - off) * es);
        if (!SPLIT && pipe)
            apply_run_pipe<F, F == HH_FMT_FP64 ? 4 : 8>(rn, rs, (uint32_t)row * es, coef, acc);
        else
            apply_run<F, 1, SPLIT, UB>(rn, rs, (uint32_t)row * es, coef, 1, 0, 1, g, G, acc);
        rn = nx;
    }
}

// One continuum run on a lane's 4 rows: columns in batches of 8 (SPLIT: the
// wave's groups take every G-th column), then clamped batches of 4.
template <int W, bool SPLIT>
__device__ inline void apply_run_cont(const Run& rn, rsrc_t rs, uint32_t off, uint32_t sh,
                                      const double* coef, int g, int G, double acc[4][1]) {
    const uint32_t cb = (uint32_t)rn.stride * 4u;        // continuum stride is in dwords
    const int n = rn.ncols;
    const int step = SPLIT ? G : 1;
    int c = SPLIT ? g : 0;
    constexpr int U = SPLIT || W > 24 ? 4 : 8;
    for (; c + (U - 1) * step < n; c += U * step) {
        CRaw<W> raw[U];
        double cf[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int cc = c + u * step;
            raw[u] = cload<W, CP_STREAM>(rs, off + (uint32_t)cc * cb);
            cf[u] = SPLIT ? ldg<double>(coef + rn.toff + cc) : ldc<double>(coef + rn.toff + cc);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double v[4];
            cwiden<W>(raw[u], sh, v);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q][0] = fma(v[q], cf[u], acc[q][0]);
        }
    }
    for (; c < n; c += 4 * step) {
        CRaw<W> raw[4];
        double cf[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int cu = c + u * step;
            const int cc = cu < n ? cu : n - 1;
            raw[u] = cload<W, CP_STREAM>(rs, off + (uint32_t)cc * cb);
            const double w = SPLIT ? ldg<double>(coef + rn.toff + cc) : ldc<double>(coef + rn.toff + cc);
            cf[u] = cu < n ? w : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double v[4];
            cwiden<W>(raw[u], sh, v);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q][0] = fma(v[q], cf[u], acc[q][0]);
        }
    }
}

template <bool SPLIT>
struct RunCont {
    Run rn;
    rsrc_t rs;
    int64_t crow;            // first row of the lane inside the cluster's columns
    const double* coef;
    int g, G;
    double (*acc)[1];
    template <int W>
    __device__ void operator()() const {
        uint32_t off, sh;
        cpos<W>(crow, off, sh);
        apply_run_cont<W, SPLIT>(rn, rs, off, sh, coef, g, G, acc);
    }
};

template <bool SPLIT>
__device__ inline void unit_runs_cont(const Desc& D, const UnitTask& ut, int b, int e, int64_t row,
                                      int g, int G, double acc[4][1]) {
    for (int i = b; i < e; ++i) {
        const Run rn = ldrec<Run>(D.uruns + i);
        const rsrc_t rs = make_rsrc(rn.base, (int64_t)rn.ncols * rn.stride * 4);
        with_width(rn.w, RunCont<SPLIT>{rn, rs, ut.poff - rn.pc + row, D.tb, g, G, acc});
    }
}

template <bool SPLIT, int UB, int FAM>
__device__ inline void unit_runs(const Desc& D, const UnitTask& ut, int64_t row, int g, int G,
                                 double acc[4][1], bool pipe) {
    unit_runs_fmt<HH_FMT_FP64, SPLIT, UB>(D, ut, ut.rb, ut.fe[0], row, g, G, acc, pipe);
    if constexpr (FAM == FAM_CONT) {
        unit_runs_cont<SPLIT>(D, ut, ut.fe[3], ut.fe[4], row, g, G, acc);
    } else {
        unit_runs_fmt<HH_FMT_FP32, SPLIT, UB>(D, ut, ut.fe[0], ut.fe[1], row, g, G, acc, pipe);
        unit_runs_fmt<HH_FMT_FP16, SPLIT, UB>(D, ut, ut.fe[1], ut.fe[2], row, g, G, acc, pipe);
        unit_runs_fmt<HH_FMT_BF16, SPLIT, UB>(D, ut, ut.fe[2], ut.fe[3], row, g, G, acc, pipe);
        if constexpr (FAM == FAM_Q43)
            unit_runs_fmt<HH_FMT_Q43, SPLIT, UB>(D, ut, ut.fe[3], ut.fe[4], row, g, G, acc, pipe);
    }
}

// Four units per workgroup, one per wave; the waves never synchronise.
template <int UB, bool PIPE, int FAM>
__device__ inline void unit_body(Desc d, const Desc* descs, const UnitTask* units, int64_t nunits) {
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int64_t ui = (int64_t)blockIdx.x * 4 + wave;
    if (ui >= nunits) return;
    const UnitTask ut = ldrec<UnitTask>(units + ui);
    const Desc D = descs ? ldrec<Desc>(descs + ut.hid) : d;
    const int P = ut.P;
    // strips of 256 rows, then one strip for the remaining rows sized to them:
    // lps lanes per 4-row group cover them, and the 64 / lps groups of the wave
    // share out the columns, so a leaf a little above 256 rows does not pay a
    // second full pass over its runs for a few rows
    for (int jlo = 0; jlo < P;) {
        const int rem = P - jlo;
        int lps = 1;
        while (lps < 64 && 4 * lps < rem) lps <<= 1;
        const int G = 64 / lps, g = lane / lps, sl = lane % lps;
        const int strip = 4 * lps;
        const int prow = jlo + 4 * sl;
        const int64_t row = prow < P ? prow : 0;     // clamped: in bounds, never written
        double acc[4][1] = {{0.0}, {0.0}, {0.0}, {0.0}};
        if (G == 1) unit_runs<false, UB, FAM>(D, ut, row, 0, 1, acc, PIPE);
        else unit_runs<true, UB, FAM>(D, ut, row, g, G, acc, PIPE);
        for (int off = lps; off < 64; off <<= 1)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q][0] += __shfl_xor(acc[q][0], off, 64);
        if (g == 0)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (prow + q < P) stg<double>(D.part + ut.po + prow + q, acc[q][0]);
        jlo += strip;
    }
}

#define HH_UNIT_KERNEL(NAME, UB, W, PIPE, FAM)                                               \
    __global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void NAME(         \
        Desc d, const Desc* descs, const UnitTask* units, int64_t nunits) {                    \
        unit_body<UB, PIPE, FAM>(d, descs, units, nunits);                                      \
    }
HH_UNIT_KERNEL(unit_kernel, 16, 4, true, FAM_FIX)
HH_UNIT_KERNEL(unitc_kernel, 16, 4, true, FAM_CONT)
HH_UNIT_KERNEL(unitq_kernel, 16, 4, true, FAM_Q43)

// y rows of one leaf: its units' partials in unit order, written in caller
// order. Lane l owns rows 4l..4l+3 of each 256-row strip.
__global__ __launch_bounds__(256) void finish_kernel(Desc d, const Desc* descs,
                                                     const FinishTask* fin, int64_t nfin) {
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int64_t fi = (int64_t)blockIdx.x * 4 + wave;
    if (fi >= nfin) return;
    const FinishTask ft = ldrec<FinishTask>(fin + fi);
    const Desc D = descs ? ldrec<Desc>(descs + ft.hid) : d;
    const int P = ft.P;
    for (int jlo = 0; jlo < P; jlo += 256) {
        const int prow = jlo + 4 * lane;
        double acc[4][1] = {{0.0}, {0.0}, {0.0}, {0.0}};
        if (prow < P)
            for (int k = 0; k < ft.nu; ++k) {
                const double* pp = D.part + ft.po + (int64_t)k * P + prow;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q][0] += ldg<double>(pp + q);
            }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (prow + q >= P) continue;
            const int64_t u = ldg<int64_t>(D.pmap + ft.poff + prow + q);
            if (u < 0) continue;
            if (D.io == HH_IO_F64) stg<double>(static_cast<double*>(D.y) + u, acc[q][0]);
            else stg<float>(static_cast<float*>(D.y) + u, (float)acc[q][0]);
        }
    }
}

// ------------------------------------------- several right-hand sides: MFMA
// v_mfma_f64_16x16x4f64: D (16 x 16) += A (16 x 4) B (4 x 16). Lane l holds
// A[l & 15][l >> 4], B[l >> 4][l & 15] and D[4 r + (l >> 4)][l & 15] in its
// register r. The reduction index K may be permuted freely as long as A and B
// use the same permutation; both kernels below let a lane hold four
// consecutive stored rows (one 16-byte load) and spend them on four MFMAs.
typedef double dbl4_t __attribute__((ext_vector_type(4)));

__device__ inline dbl4_t mfma16(double a, double b, dbl4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Coefficient of tile column cm for right-hand side rhs: at toff + cm with the
// tile's exponent, or (panel tiles) where the column map sends it.
template <bool PANEL>
__device__ inline void dotm_store(const DotTask& t, const Desc& D, int R, int cm, int rhs, double v) {
    int64_t idx = t.toff + cm;
    int e = t.exp;
    if (PANEL) {
        const int64_t m = ldg<int64_t>(t.cmap + cm);
        idx = m & (((int64_t)1 << 40) - 1);
        e = (int)(m >> 40) - 1024;
    }
    stg<double>(D.tb + idx * (int64_t)R + rhs, ldexp(v, e));
}

// Phase V: T[c][r] = 2^e sum_p V[p][c] x[p][r] for a tile of up to 16 MT
// columns of one block (MT column tiles of 16 share every x load) and NT tiles
// of 16 right-hand sides (group g). K step = 16 rows: lane (i, k) loads rows
// p0 + 4k .. p0 + 4k + 3 of column i of each column tile; MFMA m uses row
// p0 + 4k + m for the lane's k. Rows past P and columns past the tile are
// clamped in bounds with weight zero / discarded.
template <int FMT, int NT, int MT>
__device__ void dotm_tile(const DotTask& t, const Desc& D, int R, int g, int lane) {
    constexpr uint32_t es = elem_bytes<FMT>();
    const int i = lane & 15, kq = lane >> 4;
    const int P = t.P;
    // one wave-uniform descriptor for the tile; the column goes into the
    // lane's offset (a per-lane descriptor would make every load a loop over
    // the distinct descriptors of the wave)
    const rsrc_t rs = make_rsrc(t.col0, (int64_t)t.ncols * P * es);
    uint32_t cofs[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int c = 16 * mt + i < t.ncols ? 16 * mt + i : t.ncols - 1;
        cofs[mt] = (uint32_t)c * (uint32_t)P * es;
    }
    const double* xb = D.xt + t.xoff * (int64_t)R;
    int rr[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int r = 16 * (g * NT + u) + i;
        rr[u] = r < R ? r : R - 1;
    }
    // AC independent partial sums per tile pair keep the MFMA chains apart;
    // they are added in a fixed order at the end
    constexpr int AC = NT * MT >= 4 ? 1 : 4 / (NT * MT);
    dbl4_t acc[AC][MT][NT];
#pragma unroll
    for (int h = 0; h < AC; ++h)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[h][mt][u] = dbl4_t{0.0, 0.0, 0.0, 0.0};
    constexpr int KU = NT * MT == 1 ? 4 : (NT * MT == 2 || MT == 4) ? 2 : 1;
    for (int p0 = 0; p0 < P; p0 += 16 * KU) {
        double a[KU][MT][4];
        double b[KU][4][NT];
        bool pok[KU];
#pragma unroll
        for (int s = 0; s < KU; ++s) {
            const int p = p0 + 16 * s + 4 * kq;
            pok[s] = p < P;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                widen4<FMT, double>(bload4<FMT>(rs, cofs[mt] + (uint32_t)(pok[s] ? p : 0) * es), a[s][mt]);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    b[s][m][u] = ldg<double>(xb + (int64_t)(pok[s] ? p + m : 0) * R + rr[u]);
        }
#pragma unroll
        for (int s = 0; s < KU; ++s)
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const double am = pok[s] ? a[s][mt][m] : 0.0;
#pragma unroll
                    for (int u = 0; u < NT; ++u)
                        acc[m % AC][mt][u] = mfma16(am, b[s][m][u], acc[m % AC][mt][u]);
                }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = acc[0][mt][u][r];
#pragma unroll
                for (int h = 1; h < AC; ++h) v += acc[h][mt][u][r];
                const int cm = 16 * mt + 4 * r + kq, rhs = 16 * (g * NT + u) + i;
                if (cm < t.ncols && rhs < R) dotm_store<MT == DOTP_MT>(t, D, R, cm, rhs, v);
            }
}

// The same tile over continuum columns (exponent sum 0): lane (i, k) decodes
// rows p .. p + 3 of column i of each column tile.
template <int W, int NT, int MT>
__device__ void dotm_tile_cont(const DotTask& t, const Desc& D, int R, int g, int lane) {
    const int i = lane & 15, kq = lane >> 4;
    const int P = t.P;
    const int64_t cb = cont_col_bytes(P, W);
    const rsrc_t rs = make_rsrc(t.col0, (int64_t)t.ncols * cb);   // wave-uniform (see dotm_tile)
    uint32_t cofs[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int c = 16 * mt + i < t.ncols ? 16 * mt + i : t.ncols - 1;
        cofs[mt] = (uint32_t)c * (uint32_t)cb;
    }
    const double* xb = D.xt + t.xoff * (int64_t)R;
    int rr[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int r = 16 * (g * NT + u) + i;
        rr[u] = r < R ? r : R - 1;
    }
    constexpr int AC = NT * MT >= 4 ? 1 : 4 / (NT * MT);
    dbl4_t acc[AC][MT][NT];
#pragma unroll
    for (int h = 0; h < AC; ++h)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[h][mt][u] = dbl4_t{0.0, 0.0, 0.0, 0.0};
    for (int p0 = 0; p0 < P; p0 += 16) {
        const int p = p0 + 4 * kq;
        const bool pok = p < P;
        uint32_t off, sh;
        cpos<W>(pok ? p : 0, off, sh);
        double a[MT][4];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) cwiden<W>(cload<W>(rs, cofs[mt] + off), sh, a[mt]);
        double b[4][NT];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int u = 0; u < NT; ++u) b[m][u] = ldg<double>(xb + (int64_t)(pok ? p + m : 0) * R + rr[u]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const double am = pok ? a[mt][m] : 0.0;
#pragma unroll
                for (int u = 0; u < NT; ++u)
                    acc[m % AC][mt][u] = mfma16(am, b[m][u], acc[m % AC][mt][u]);
            }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = acc[0][mt][u][r];
#pragma unroll
                for (int h = 1; h < AC; ++h) v += acc[h][mt][u][r];
                const int cm = 16 * mt + 4 * r + kq, rhs = 16 * (g * NT + u) + i;
                if (cm < t.ncols && rhs < R) dotm_store<MT == DOTP_MT>(t, D, R, cm, rhs, v);
            }
}

template <int NT, int MT>
struct DotmCont {
    DotTask t;
    Desc D;
    int R, g, lane;
    template <int W>
    __device__ void operator()() const { dotm_tile_cont<W, NT, MT>(t, D, R, g, lane); }
};

// Tiles x right-hand-side groups, four per workgroup (one per wave); the groups
// of one tile are neighbours, so its columns are read from HBM about once.
template <int NT, int FAM, int MT>
__global__ __launch_bounds__(256) void dotm_kernel(Desc d, const Desc* descs, const DotTask* tiles,
                                                   int64_t ntiles, int R, int ngroups) {
    constexpr bool CONT = FAM == FAM_CONT;
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + wave;
    if (item >= ntiles * ngroups) return;
    const int64_t ti = item / ngroups;
    const int g = (int)(item - ti * ngroups);
    const DotTask t = ldrec<DotTask>(tiles + ti);
    const Desc D = descs ? ldrec<Desc>(descs + t.hid) : d;
    if (CONT && t.fmt == HH_FMT_CONT) {
        if constexpr (CONT) with_width(t.w, DotmCont<NT, MT>{t, D, R, g, lane});
        return;
    }
    if constexpr (FAM == FAM_Q43) {
        if (t.fmt == HH_FMT_Q43) {
            dotm_tile<HH_FMT_Q43, NT, MT>(t, D, R, g, lane);
            return;
        }
    }
    switch (t.fmt) {
        case HH_FMT_FP64: dotm_tile<HH_FMT_FP64, NT, MT>(t, D, R, g, lane); break;
        case HH_FMT_FP32: dotm_tile<HH_FMT_FP32, NT, MT>(t, D, R, g, lane); break;
        case HH_FMT_FP16: dotm_tile<HH_FMT_FP16, NT, MT>(t, D, R, g, lane); break;
        default: dotm_tile<HH_FMT_BF16, NT, MT>(t, D, R, g, lane); break;
    }
}

// Phase U for 64 rows of a leaf (four 16-row subtiles q: rows base + 4 i + q)
// and NT tiles of right-hand sides: lane (i, k) loads rows base + 4i .. + 3 of
// column c + k, one row per subtile; K step = 4 columns, four steps per pass.
// SLOT: the format's slot in the cluster's run list.
template <int F, int NT, int SLOT = F>
__device__ inline void accm_runs(const Desc& D, int64_t ci, const LeafTask& lt, int rowbase, int R,
                                 int g, int lane, dbl4_t acc[4][NT]) {
    constexpr uint32_t es = elem_bytes<F>();
    const int i = lane & 15, kq = lane >> 4;
    const int row0 = rowbase + 4 * i;
    const uint32_t voff = (uint32_t)(row0 < lt.P ? row0 : 0) * es;
    int rr[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int r = 16 * (g * NT + u) + i;
        rr[u] = r < R ? r : R - 1;
    }
    const int rb = ldc<int32_t>(D.cl_run + NFMT * ci + SLOT), re = ldc<int32_t>(D.cl_run + NFMT * ci + SLOT + 1);
    for (int ri = rb; ri < re; ++ri) {
        const Run rn = ldrec<Run>(D.runs + ri);
        const double* coef = rn.from_x ? D.xt : D.tb;
        const int64_t off = lt.poff - rn.pc;
        const rsrc_t rs = make_rsrc(static_cast<const char*>(rn.base) + off * es,
                                    ((int64_t)rn.ncols * rn.stride - off) * es);
        const int n = rn.ncols;
        constexpr int KS = NT >= 4 ? 2 : 4;           // K steps of 4 columns per pass
        for (int c = 0; c < n; c += 4 * KS) {
            double a[KS][4];
            double b[KS][NT];
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4) {
                const int cc = c + 4 * s4 + kq;
                const int ccl = cc < n ? cc : n - 1;
                widen4<F, double>(bload4<F>(rs, voff + (uint32_t)ccl * (uint32_t)rn.stride * es), a[s4]);
                if (cc >= n) a[s4][0] = a[s4][1] = a[s4][2] = a[s4][3] = 0.0;
#pragma unroll
                for (int u = 0; u < NT; ++u) b[s4][u] = ldg<double>(coef + ((int64_t)rn.toff + ccl) * R + rr[u]);
            }
#pragma unroll
            for (int s4 = 0; s4 < KS; ++s4)
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int u = 0; u < NT; ++u) acc[q][u] = mfma16(a[s4][q], b[s4][u], acc[q][u]);
        }
    }
}

// The same for the cluster's continuum runs (the width W is per run).
template <int W, int NT>
__device__ inline void accm_run_cont(const Run& rn, const double* tb, int64_t crow, int R, int g,
                                     int lane, dbl4_t acc[4][NT]) {
    const int i = lane & 15, kq = lane >> 4;
    int rr[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int r = 16 * (g * NT + u) + i;
        rr[u] = r < R ? r : R - 1;
    }
    const uint32_t cb = (uint32_t)rn.stride * 4u;
    const rsrc_t rs = make_rsrc(rn.base, (int64_t)rn.ncols * cb);
    uint32_t off, sh;
    cpos<W>(crow, off, sh);
    const int n = rn.ncols;
    constexpr int KS = NT >= 4 ? 2 : 4;
    for (int c = 0; c < n; c += 4 * KS) {
        double a[KS][4];
        double b[KS][NT];
#pragma unroll
        for (int s4 = 0; s4 < KS; ++s4) {
            const int cc = c + 4 * s4 + kq;
            const int ccl = cc < n ? cc : n - 1;
            cwiden<W>(cload<W>(rs, off + (uint32_t)ccl * cb), sh, a[s4]);
            if (cc >= n) a[s4][0] = a[s4][1] = a[s4][2] = a[s4][3] = 0.0;
#pragma unroll
            for (int u = 0; u < NT; ++u) b[s4][u] = ldg<double>(tb + ((int64_t)rn.toff + ccl) * R + rr[u]);
        }
#pragma unroll
        for (int s4 = 0; s4 < KS; ++s4)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int u = 0; u < NT; ++u) acc[q][u] = mfma16(a[s4][q], b[s4][u], acc[q][u]);
    }
}

template <int NT>
struct AccmCont {
    Run rn;
    const double* tb;
    int64_t crow;
    int R, g, lane;
    dbl4_t (*acc)[NT];
    template <int W>
    __device__ void operator()() const { accm_run_cont<W, NT>(rn, tb, crow, R, g, lane, acc); }
};

template <int NT>
__device__ inline void accm_runs_cont(const Desc& D, int64_t ci, const LeafTask& lt, int rowbase,
                                      int R, int g, int lane, dbl4_t acc[4][NT]) {
    const int i = lane & 15;
    const int row0 = rowbase + 4 * i;
    const int rb = ldc<int32_t>(D.cl_run + NFMT * ci + HH_FMT_CONT);
    const int re = ldc<int32_t>(D.cl_run + NFMT * ci + HH_FMT_CONT + 1);
    for (int ri = rb; ri < re; ++ri) {
        const Run rn = ldrec<Run>(D.runs + ri);
        const int64_t crow = lt.poff - rn.pc + (row0 < lt.P ? row0 : 0);
        with_width(rn.w, AccmCont<NT>{rn, D.tb, crow, R, g, lane, acc});
    }
}

// One workgroup per (leaf, right-hand-side group); wave w owns rows 64 w ..
// 64 w + 63 of each 256-row strip of the leaf; writes y in caller order.
template <int NT, int FAM>
__global__ __launch_bounds__(256) void accm_kernel(Desc d, const Desc* descs, const LeafTask* leaves,
                                                   int R, int ngroups) {
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int64_t li = blockIdx.x / ngroups;
    const int g = (int)(blockIdx.x - li * ngroups);
    const LeafTask lt = ldrec<LeafTask>(leaves + li);
    const Desc D = descs ? ldrec<Desc>(descs + lt.hid) : d;
    const int i = lane & 15, kq = lane >> 4;
    for (int strip = 0; strip < lt.P; strip += 256) {
        const int rowbase = strip + 64 * wave;
        if (rowbase >= lt.P) break;
        dbl4_t acc[4][NT];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int u = 0; u < NT; ++u) acc[q][u] = dbl4_t{0.0, 0.0, 0.0, 0.0};
        for (int l = 0; l <= D.L; ++l) {
            const int64_t ci = cluster_index(D, l, lt.leaf);
            accm_runs<HH_FMT_FP64, NT>(D, ci, lt, rowbase, R, g, lane, acc);
            accm_runs<HH_FMT_FP32, NT>(D, ci, lt, rowbase, R, g, lane, acc);
            accm_runs<HH_FMT_FP16, NT>(D, ci, lt, rowbase, R, g, lane, acc);
            accm_runs<HH_FMT_BF16, NT>(D, ci, lt, rowbase, R, g, lane, acc);
            if constexpr (FAM == FAM_CONT) accm_runs_cont<NT>(D, ci, lt, rowbase, R, g, lane, acc);
            if constexpr (FAM == FAM_Q43)
                accm_runs<HH_FMT_Q43, NT, HH_FMT_CONT>(D, ci, lt, rowbase, R, g, lane, acc);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int u = 0; u < NT; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rowbase + 4 * (4 * r + kq) + q;
                    const int rhs = 16 * (g * NT + u) + i;
                    if (row >= lt.P || rhs >= R) continue;
                    const int64_t uidx = ldg<int64_t>(D.pmap + lt.poff + row);
                    if (uidx < 0) continue;
                    if (D.io == HH_IO_F64)
                        stg<double>(static_cast<double*>(D.y) + uidx * R + rhs, acc[q][u][r]);
                    else
                        stg<float>(static_cast<float*>(D.y) + uidx * R + rhs, (float)acc[q][u][r]);
                }
    }
}

// RHS tiles of 16 per group: phase V up to four; phase U two (a group of four
// would need 128 accumulator registers and one wave per SIMD).
static inline int rhs_tiles_per_group(int R) { return R <= 16 ? 1 : R <= 32 ? 2 : 4; }
static inline int rhs_tiles_per_group_u(int R) { return R <= 16 ? 1 : 2; }

// ------------------------------------------------------------- launchers
void launch_gather(const Desc& d, const Desc* descs, int nh, int64_t max_np, int R, void* stream) {
    int64_t total = max_np * R;
    int64_t g = (total + 255) / 256;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)g, nh), dim3(256), 0, (hipStream_t)stream, d,
                       descs, R);
}

template <int FAM>
static void launch_dotm(const Desc& d, const Desc* descs, const DotTask* tasks, int64_t ntasks,
                        int R, void* stream) {
    const int nt = rhs_tiles_per_group(R);
    const int ngroups = ((R + 15) / 16 + nt - 1) / nt;
    const unsigned grid = (unsigned)((ntasks * ngroups + 3) / 4);
    if (FAM != FAM_CONT && R <= PANEL_MAX_R)
        hipLaunchKernelGGL((dotm_kernel<1, FAM == FAM_CONT ? FAM_FIX : FAM, DOTP_MT>), dim3(grid),
                           dim3(256), 0, (hipStream_t)stream, d, descs, tasks, ntasks, R, ngroups);
    else if (nt == 1)
        hipLaunchKernelGGL((dotm_kernel<1, FAM, DOTM_MT>), dim3(grid), dim3(256), 0,
                           (hipStream_t)stream, d, descs, tasks, ntasks, R, ngroups);
    else if (nt == 2)
        hipLaunchKernelGGL((dotm_kernel<2, FAM, DOTM_MT>), dim3(grid), dim3(256), 0,
                           (hipStream_t)stream, d, descs, tasks, ntasks, R, ngroups);
    else
        hipLaunchKernelGGL((dotm_kernel<4, FAM, DOTM_MT>), dim3(grid), dim3(256), 0,
                           (hipStream_t)stream, d, descs, tasks, ntasks, R, ngroups);
}

void launch_dot(const Desc& d, const Desc* descs, const DotTask* tasks, int64_t ntasks, int R,
                int fam, void* stream) {
    if (ntasks <= 0) return;
    if (R == 1) {
        if (fam == FAM_CONT)
            hipLaunchKernelGGL(dot1c_kernel, dim3((unsigned)ntasks), dim3(256), 0, (hipStream_t)stream,
                               d, descs, tasks);
        else if (fam == FAM_Q43)
            hipLaunchKernelGGL(dot1q_kernel, dim3((unsigned)ntasks), dim3(256), 0, (hipStream_t)stream,
                               d, descs, tasks);
        else
            hipLaunchKernelGGL(dot1_kernel, dim3((unsigned)ntasks), dim3(256), 0, (hipStream_t)stream,
                               d, descs, tasks);
        return;
    }
    // several right-hand sides: panel tiles (up to PANEL_MAX_R right-hand
    // sides, no continuum blocks), else tiles of at most 16 columns
    if (fam == FAM_CONT) launch_dotm<FAM_CONT>(d, descs, tasks, ntasks, R, stream);
    else if (fam == FAM_Q43) launch_dotm<FAM_Q43>(d, descs, tasks, ntasks, R, stream);
    else launch_dotm<FAM_FIX>(d, descs, tasks, ntasks, R, stream);
}

void launch_dot1_panel(const Desc& d, const Desc* descs, const DotTask* tasks, int64_t ntasks,
                       int fam, void* stream) {
    if (ntasks <= 0) return;
    if (fam == FAM_Q43)
        hipLaunchKernelGGL(dot1pq_kernel, dim3((unsigned)ntasks), dim3(256), 0, (hipStream_t)stream, d,
                           descs, tasks);
    else
        hipLaunchKernelGGL(dot1p_kernel, dim3((unsigned)ntasks), dim3(256), 0, (hipStream_t)stream, d,
                           descs, tasks);
}

template <int FAM>
static void launch_accm(const Desc& d, const Desc* descs, const LeafTask* leaves, int64_t nleaves,
                        int R, void* stream) {
    const int nt = rhs_tiles_per_group_u(R);
    const int ngroups = ((R + 15) / 16 + nt - 1) / nt;
    const unsigned grid = (unsigned)(nleaves * ngroups);
    if (nt == 1)
        hipLaunchKernelGGL((accm_kernel<1, FAM>), dim3(grid), dim3(256), 0, (hipStream_t)stream, d,
                           descs, leaves, R, ngroups);
    else
        hipLaunchKernelGGL((accm_kernel<2, FAM>), dim3(grid), dim3(256), 0, (hipStream_t)stream, d,
                           descs, leaves, R, ngroups);
}

void launch_accumulate(const Desc& d, const Desc* descs, const LeafTask* leaves, int64_t nleaves,
                       int R, int fam, void* stream) {
    if (nleaves <= 0) return;
    if (fam == FAM_CONT) launch_accm<FAM_CONT>(d, descs, leaves, nleaves, R, stream);
    else if (fam == FAM_Q43) launch_accm<FAM_Q43>(d, descs, leaves, nleaves, R, stream);
    else launch_accm<FAM_FIX>(d, descs, leaves, nleaves, R, stream);
}

void launch_units(const Desc& d, const Desc* descs, const UnitTask* units, int64_t nunits,
                  const FinishTask* fin, int64_t nfin, int fam, void* stream) {
    if (nunits > 0) {
        const dim3 grid((unsigned)((nunits + 3) / 4));
        if (fam == FAM_CONT)
            hipLaunchKernelGGL(unitc_kernel, grid, dim3(256), 0, (hipStream_t)stream, d, descs, units,
                               nunits);
        else if (fam == FAM_Q43)
            hipLaunchKernelGGL(unitq_kernel, grid, dim3(256), 0, (hipStream_t)stream, d, descs, units,
                               nunits);
        else
            hipLaunchKernelGGL(unit_kernel, grid, dim3(256), 0, (hipStream_t)stream, d, descs, units,
                               nunits);
    }
    if (nfin > 0)
        hipLaunchKernelGGL(finish_kernel, dim3((unsigned)((nfin + 3) / 4)), dim3(256), 0,
                           (hipStream_t)stream, d, descs, fin, nfin);
}

}  // namespace hh
