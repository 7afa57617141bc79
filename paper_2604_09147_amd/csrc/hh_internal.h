// Internal data structures of the H_h library (host and device).
#pragma once

#include <cstdint>
#include <array>
#include <string>
#include <vector>

#include "../../include/hh.h"

namespace hh {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
struct Error {
    hh_status code;
    std::string msg;
};
[[noreturn]] void fail(hh_status code, const std::string& msg);

// ------------------------------------------------------------------- plan
// Tree of Sec. 2.1 and the block partition of Alg. 1 (host only).
struct Blk {
    int32_t level, kind;
    int64_t bi, bj;          // Morton box indices at `level`
    int64_t ib, ie, jb, je;  // tree-order row / column ranges
};

struct Plan {
    int64_t n = 0;
    int d = 0, L = 0, ell = 0, leaf_size = 0;
    double eta = 0;
    std::vector<int64_t> perm;                 // tree position -> caller index
    std::vector<std::vector<int64_t>> ranges;  // per level: 2 * 2^(d l) [beg, end)
    std::vector<Blk> blocks;                   // canonical order (level, bi, bj)
};

Plan make_plan(const double* pts, int64_t n, int d, double eta, int switch_level,
               int leaf_size);
bool adm_s(const int64_t* ci, const int64_t* cj, int d, double eta);
void box_coords(int64_t box, int level, int d, int64_t* c);

// --------------------------------------------------------- device layouts
// Padded tree coordinates: every leaf occupies round_up(n_leaf, 4) slots so
// that a wave lane owning 4 consecutive rows always reads aligned vectors.
constexpr int ROW_PAD = 4;

// Storage formats of the low-rank factors: HH_FMT_FP64 .. HH_FMT_BF16, the
// continuum format HH_FMT_CONT (per block t fraction bits, 9 + t bits per
// entry, entries packed back to back in every column) and the 8-bit
// HH_FMT_Q43 (NFMT_CODES format codes). A handle stores continuum or q43
// blocks, never both, so the run lists keep NFMT slots per cluster and q43
// runs take the continuum slot.
constexpr int NFMT_CODES = 6;
constexpr int NFMT = 5;
constexpr int fmt_slot(int fmt) { return fmt == HH_FMT_Q43 ? HH_FMT_CONT : fmt; }
// q43 codes are widened in the product kernels by moving their bits into an
// fp16 (sign to bit 15, exponent field E to bits 10..14, fraction f to bits
// 7..9): an fp16 has 8 more exponent bias than q43, so its value is the q43
// value times 2^-8 for every code, subnormals included. The two factors of a
// block thus carry 2^-16, which the block's coefficient scale takes back.
constexpr int fmt_exp_bias(int fmt) { return fmt == HH_FMT_Q43 ? 16 : 0; }
// Bytes of one continuum column of P entries of w bits: whole 16-byte units,
// so every column starts 16-byte aligned (constexpr: usable in device code).
constexpr int64_t cont_col_bytes(int64_t P, int w) {
    return ((P * w + 127) >> 7) << 4;
}

struct Run;

// Per-handle device pointers the product kernels need for one direction of the
// product (passed by value, or as an array indexed by DotTask::hid /
// LeafTask::hid in a batched launch).
struct Desc {
    double* xt;              // gathered x, padded tree order, NP x R (row-major)
    double* tb;              // column coefficients, C x R (row-major)
    const int64_t* pmap;     // padded slot -> caller index (-1 = pad), NP entries
    const void* x;           // caller x (N x R)
    void* y;                 // caller y (N x R)
    const Run* runs;         // runs of every cluster, clusters in (level, box) order
    const int32_t* cl_run;   // runs of cluster c in format f: [cl_run[NFMT c + f], cl_run[NFMT c + f + 1])
    const Run* uruns;        // runs of the single-vector work units
    double* part;            // partial sums of the work units
    int64_t np;              // padded length
    int32_t io;              // HH_IO_F64 / HH_IO_F32
    int32_t d, L;            // dimension and depth of the tree
    int32_t pad_;
};

// Inner products of stored columns with a slice of the gathered vector:
// tb[toff + c] = sum_j col_c[j] xt[xoff + j]  for c < ncols, j < P.
// The coefficient carries the block's factor scales: tb = 2^exp (col . xt).
struct DotTask {
    const void* col0;        // first element of column 0; column c starts c * P elements
                             // later (continuum: c * cont_col_bytes(P, w) bytes later)
    int64_t xoff;            // padded row offset of the slice of xt
    int64_t toff;            // coefficient index of column 0
    int32_t P;               // column length (padded rows, multiple of 4)
    int32_t ncols;
    int32_t fmt;             // HH_FMT_*
    int32_t hid;             // handle index in a batched launch
    int32_t exp;             // eU + eV (power-of-two factor scales, exact)
    int32_t w;               // continuum: bits per stored entry (9 + t); else 0
    // Panel tiles (columns of several blocks stored one after another): per
    // column c, cmap[c] = coefficient index | (exponent + 1024) << 40, used
    // instead of toff + c and exp; null for the columns of one block.
    const int64_t* cmap;
};

// Columns stored with a common stride and consecutive coefficients, restricted
// to the rows of a cluster: the columns of one block, or of several blocks of
// the same cluster and format stored one after another (their factors are
// laid out that way). Applied to a leaf inside the cluster:
// y_leaf += sum_c col_c[leaf rows] coef_c with coef_c = tb[toff + c]
// (low-rank, scales already in tb) or xt[toff + c] (dense block).
struct Run {
    const void* base;        // element (cluster row 0, column 0)
    int64_t pc;              // padded offset of the cluster's first row
    int32_t stride;          // elements between consecutive columns
    int32_t toff;
    int32_t ncols;
    int16_t w;               // continuum: bits per stored entry (9 + t); else 0
    int8_t fmt;              // HH_FMT_*; dense blocks are HH_FMT_FP64
    int8_t from_x;
};

// One nonempty leaf box (one wave of the accumulation kernel).
struct LeafTask {
    int64_t poff;            // padded offset of the leaf
    int32_t P;               // padded rows of the leaf
    int32_t leaf;            // Morton index of the leaf box at level L
    int32_t hid;             // handle index in a batched launch
    int32_t pad_;
};

// A slice of one leaf's runs (one wave of the single-vector accumulation).
// Its runs in the unit run list are grouped by format: fp64 [rb, fe[0]),
// fp32 [fe[0], fe[1]), fp16 [fe[1], fe[2]), bf16 [fe[2], fe[3]), continuum
// or q43 [fe[3], fe[4]). The wave writes its partial sum of the leaf's rows to
// part[po .. po + P).
struct UnitTask {
    int64_t poff;            // padded offset of the leaf
    int64_t po;              // offset of the unit's partial rows
    int32_t P;               // padded rows of the leaf
    int32_t rb;
    int32_t fe[NFMT];
    int32_t hid;             // handle index in a batched launch
};

// One leaf of the finishing kernel: y rows = sum over its nu units of
// part[po + k P + row].
struct FinishTask {
    int64_t poff;
    int64_t po;
    int32_t P;
    int32_t leaf;            // Morton index of the leaf box
    int32_t nu;
    int32_t hid;
};

// Host record of one block after the build.
struct BlockRec {
    Blk b;
    int32_t rank = 0, fmt = HH_FMT_FP64, eU = 0, eV = 0;
    int32_t t = 0;                    // fraction bits when fmt == HH_FMT_CONT
    bool lowrank = false;
    double nb2 = 0, entry2 = 0, tail_prev = 0, tail = 0;
    const void* u_ptr = nullptr;      // stored factors (format fmt), padded-row layout
    const void* v_ptr = nullptr;
    const double* d_ptr = nullptr;    // dense block, PI x n column-major
    const double* dt_ptr = nullptr;   // its transpose, PJ x m column-major (product with H^T)
    int64_t col = -1;                 // coefficient index of column 0 (product with H)
    int64_t col_t = -1;               // coefficient index of column 0 (product with H^T)
    int64_t PI = 0, PJ = 0;           // padded lengths of row / column clusters
    int64_t pI = 0, pJ = 0;           // padded offsets of row / column clusters
};

// Columns per several-RHS phase-V tile: DOTM_MT MFMA tiles of 16 columns.
constexpr int DOTM_MT = 1;
// Up to PANEL_MAX_R right-hand sides, phase V of handles without continuum
// blocks runs on panel tiles instead: DOTP_MT x 16 consecutive stored columns
// of blocks that share the column cluster, format and stride (one x_J load
// serves all of them).
constexpr int DOTP_MT = 4;
constexpr int PANEL_MAX_R = 16;

// Storage family of a launch (the kernel variant): the fixed formats, the
// continuum format with fp64, or the fixed formats with q43.
enum { FAM_FIX = 0, FAM_CONT = 1, FAM_Q43 = 2 };

// Kernel launch wrappers (defined in the .hip files). fam: the storage family
// of the handle (of every handle of a batch).
void launch_gather(const Desc& d, const Desc* descs, int nh, int64_t max_np, int R, void* stream);
void launch_dot(const Desc& d, const Desc* descs, const DotTask* tasks, int64_t ntasks,
                int R, int fam, void* stream);
// One right-hand side over panel tasks (DotTask::cmap set); fam FAM_FIX or FAM_Q43.
void launch_dot1_panel(const Desc& d, const Desc* descs, const DotTask* tasks, int64_t ntasks,
                       int fam, void* stream);
void launch_accumulate(const Desc& d, const Desc* descs, const LeafTask* leaves, int64_t nleaves,
                       int R, int fam, void* stream);
void launch_units(const Desc& d, const Desc* descs, const UnitTask* units, int64_t nunits,
                  const FinishTask* fin, int64_t nfin, int fam, void* stream);

}  // namespace hh

struct hh_plan {
    hh::Plan p;
};
