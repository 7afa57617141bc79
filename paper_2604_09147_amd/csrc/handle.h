// The opaque handle behind hh_handle*.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "hh_build.h"
#include "hh_internal.h"

namespace hh {

// Owned device allocation list; freed by the handle.
struct DevMem {
    std::vector<void*> ptrs;
    void* alloc(size_t bytes, bool zero = true);
    void release(void* p);
    void free_all();
    ~DevMem() { free_all(); }
};

struct TaskSet {                      // one direction of the product
    std::vector<DotTask> dot;
    std::vector<DotTask> dotm;        // tiles of at most 16 columns (several RHS)
    std::vector<DotTask> dotp;        // panel tiles (2 .. PANEL_MAX_R right-hand sides)
    std::vector<DotTask> dot1p;       // panel tasks of one right-hand side
    bool dot_panel = false;           // one right-hand side runs phase V on dot1p
    std::vector<int64_t> pcols;       // their column maps (DotTask::cmap)
    std::vector<LeafTask> leaf;
    std::vector<UnitTask> unit;       // single-vector work units, leaf by leaf
    std::vector<Run> uruns;           // their runs, format-grouped per unit
    std::vector<FinishTask> fin;      // one per nonempty leaf
    std::vector<Run> runs;            // grouped by cluster, clusters in (level, box) order
    std::vector<int32_t> cl_run;      // NFMT (sum_l 2^(d l)) + 1 boundaries (cluster, format)
    DotTask* d_dot = nullptr;
    DotTask* d_dotm = nullptr;
    DotTask* d_dotp = nullptr;
    DotTask* d_dot1p = nullptr;
    int64_t* d_pcols = nullptr;
    LeafTask* d_leaf = nullptr;
    UnitTask* d_unit = nullptr;
    Run* d_uruns = nullptr;
    FinishTask* d_fin = nullptr;
    Run* d_runs = nullptr;
    int32_t* d_cl_run = nullptr;
};

}  // namespace hh

struct hh_handle {
    hh::Plan plan;
    int device = 0;
    hh::KernelDev kd{};
    double tol = 0;
    hh_options opt{};
    std::vector<hh::BlockRec> blocks;
    // padded layout
    int64_t np = 0;
    std::vector<int64_t> leaf_poff, leaf_psz, tpad;
    // device data
    hh::DevMem mem;
    double* d_pts = nullptr;
    double* d_nrm = nullptr;
    int64_t* d_tpad = nullptr;
    int64_t* d_pmap = nullptr;
    hh::TaskSet fwd, bwd;
    int64_t ncols = 0;
    // product workspace
    double* xt = nullptr;
    double* tb = nullptr;
    int64_t ws_R = 0;
    double* part = nullptr;           // partial rows of the work units (both directions)
    int64_t part_rows = 0;
    int64_t part_cap = 0;             // rows the part buffer holds
    // task-table parameters (hh_options / hh_autotune)
    int64_t unit_bytes = 0;           // factor bytes per single-vector work unit
    int64_t dot_task_elems = 0;       // stored elements per single-vector phase-V task
    // fp64 factors kept when every low-rank block is stored in fp64
    bool all_fp64 = false;
    bool has_cont = false;            // some block stored in the continuum format
    int family = 0;                   // FAM_*: the product kernels' storage family
    hh_stats stats{};
};
