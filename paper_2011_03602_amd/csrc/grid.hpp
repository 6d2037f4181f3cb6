// The grid handle: the CPU program's variables (borrowed host arrays), their
// device copies, the offload gene and the validity state the planner works on.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "abi_util.hpp"
#include "ofl_internal.hpp"
#include "planner.hpp"

struct ofl_grid {
    int I = 0, J = 0, K = 0;
    size_t n = 0;  // I*J*K
    int fmt = OFL_COEF_F32;
    int sum_mode = OFL_SUM_F64;
    float *p = nullptr;
    float *wrk2 = nullptr;
    const float *coef[ofl::kNCoef] = {};
    void *user_stream = nullptr;
    void *arena = nullptr;
    size_t arena_bytes = 0;
    int want_device = -1;
    int row_align = 0;  // desc.row_align: 0 for 128-byte rows

    unsigned mask = OFL_MASK_ALL_GPU;
    int mode = OFL_XFER_HOISTED;
    int level[3] = {OFL_LEVEL_K, OFL_LEVEL_K, OFL_LEVEL_K};  // where each GPU nest's region opens
    ofl::TileCfg tile;
    bool tile_chosen = false;  // set by ofl_set_tile or the tuner; else the default follows the fusion
    bool in_region = false;
    ofl::Validity valid = ofl::fresh_validity();

    // bfloat16 formats: encoded host copies of the read-only arrays + biases
    std::vector<uint16_t> enc[ofl::kNCoef];
    float bias[ofl::kNCoef] = {};

    // device side (created on first GPU use)
    bool dev_ready = false;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *block = nullptr;
    bool own_block = false;
    ofl::Layout lay;
    ofl::GridView view{};
    bool pending = false;  // device work issued since the last synchronisation

    bool gosa_on_dev = false;
    double gosa_host = 0.0;

    ofl_stats stats{};
    bool profiling = false;
    unsigned prof_nests = OFL_MASK_ALL_GPU;  // nests whose GPU runs are bracketed by events
    bool prof_open = false;                  // the current nest recorded its start event
    std::vector<hipEvent_t> ev;   // pairs (start, end)
    std::vector<int> ev_nest;     // nest of each pair in use
    size_t ev_used = 0;

    // fusion of adjacent GPU nests (gene 111, hoisted): OFL_FUSE_* bits
    unsigned fusion = 0;
    double *fused_parts = nullptr;   // one FP64 partial per sweep wave
    long long fused_parts_cap = 0;
    bool wrk2_boundary_ok = false;   // device wrk2 carries p's boundary (needed before swapping)
    unsigned swap_epoch = 0;         // bumped whenever p and wrk2 exchange device buffers

    // residual nests split into regions: one FP64 sum per region
    double *region_sums = nullptr;
    long long region_sums_cap = 0;
    std::vector<double> region_host;  // per-iteration placement: the sums brought home

    // A search stops a run that outlives its time limit (steady clock, ns; 0 = none).
    long long deadline_ns = 0;

    // Steady-state iterations replayed from captured HIP graphs (whole nests,
    // hoisted, every nest on the GPU): two cached graphs, one per length.
    struct LoopGraph {
        hipGraphExec_t exec = nullptr;
        ofl::GridView view{};
        ofl::TileCfg tile;
        float omega = 0.f;
        int iters = 0;
        bool whole_rows = false;
    };
    LoopGraph graphs[2];
    int graph_next = 0;  // slot the next capture replaces

    bool broken = false;
    int batch_refs = 0;
};

namespace ofl {

// Thrown by a run that passed its grid's deadline (never crosses the C interface:
// only a search sets deadlines, and it catches this).
struct Timeout {};

ofl::TileCfg default_tile(int I, int fmt, unsigned fusion);
bool grid_whole_nests(const ofl_grid *g);
int loop_gene_bits(const ofl_grid *g);
void decode_loop_gene(const ofl_grid *g, uint32_t gene, unsigned *mask, int level[3]);
void grid_ensure_device(ofl_grid *g);
void grid_sync(ofl_grid *g);
void grid_exec(ofl_grid *g, const std::vector<Xfer> &xs);
void *grid_array_ptr(ofl_grid *g, int a);
void grid_run_loop(ofl_grid *g, int iters, float omega, int nests);
double grid_fetch_gosa(ofl_grid *g);
void grid_swap_p_wrk2(ofl_grid *g);
void grid_sync_wrk2_boundary(ofl_grid *g);

// Run f() for a grid handle: a handle that an earlier device error made
// unusable is refused (OFL_EDEVICE is sticky), and a device error raised once
// the grid's device state exists makes it so. Before that (no GPU, a failed
// first allocation) the handle stays usable, e.g. for an all-CPU gene.
template <class F>
int grid_call(ofl_grid *g, F &&f) {
    if (!g) {
        set_last_error("NULL grid handle");
        return OFL_EINVAL;
    }
    if (g->broken) {
        set_last_error("grid handle unusable after an earlier device error");
        return OFL_EDEVICE;
    }
    bool dev_err = false;
    const int rc = guarded(&dev_err, f);
    if (dev_err && g->dev_ready)
        g->broken = true;
    return rc;
}

}  // namespace ofl
