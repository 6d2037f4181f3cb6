// Batch handle: several grids run by batched kernels in one HIP graph.
#pragma once

#include <cmath>
#include <vector>

#include "grid.hpp"

struct ofl_batch {
    std::vector<ofl_grid *> grids;
    int fmt = OFL_COEF_F32;
    int sum_mode = OFL_SUM_F64;
    int device = 0;
    int cu_count = 256;
    hipStream_t stream = nullptr;
    ofl::TileCfg tile;
    bool tile_chosen = false;  // set by the caller or a search: fusion leaves it as it is

    unsigned fusion = 0;  // OFL_FUSE_* bits for the batched iterations

    bool tables_ready = false;
    void *d_views = nullptr;          // views as the grids hold them (even iterations)
    void *d_views_swapped = nullptr;  // p and wrk2 exchanged (odd iterations of a swapping run)
    void *d_fparts = nullptr;         // fused residual: two buffers (even, odd iterations) of one partial per sweep wave
    long long fparts_len = 0;         // partials per buffer
    void *d_frange = nullptr;         // per grid, its range of d_fparts (ngrids + 1 entries)
    void *d_sitems = nullptr;
    void *d_ritems = nullptr;
    void *d_range = nullptr;
    void *d_partials = nullptr;
    int s_cnt = 0;  // sweep items (every grid's, largest grid first)
    int r_cnt = 0;  // residual/copy-back items

    std::vector<int> gvec;          // per grid, its points per lane in the batch

    std::vector<int> partial_base;  // per grid, its first residual partial
    std::vector<int> nseg;          // per grid, segments per plane in packed rows (0: one row per wave)

    hipGraphExec_t exec = nullptr;
    int graph_iters = -1;
    float graph_omega = NAN;
    unsigned graph_fusion = 0;

    bool broken = false;  // a device error left the batch (and its grids) unusable
};

namespace ofl {

void batch_build_tables(ofl_batch *b);
void batch_prepare(ofl_batch *b);
void batch_enqueue(ofl_batch *b, int iters, float omega);
void batch_launch(ofl_batch *b, int iters, float omega);
void batch_finish(ofl_batch *b, int iters, double *gosa_out);
void batch_mark_done(ofl_batch *b, int iters);
void batch_after_run(ofl_batch *b, int iters);
void batch_upload_views(ofl_batch *b);
int batch_auto_vec(int I);
bool batch_packed(const ofl::Layout &L, const ofl::TileCfg &t, int *vec, int *nseg);
// A new batch's tile for coefficient format fmt and fusion bits, re-derived by
// ofl_batch_set_fusion until a tile is set or searched.
ofl::TileCfg batch_default_tile(int fmt, unsigned fusion);
int batch_auto_vec(int I);
bool batch_auto_vec_tile(const ofl_tile &t);

// Run f() for a batch handle: refused once a device error made the batch
// unusable; a device error in f marks the batch and every grid in it so, since
// their device state is then unknown (OFL_EDEVICE is sticky).
template <class F>
int batch_call(ofl_batch *b, F &&f) {
    if (!b) {
        set_last_error("NULL batch handle");
        return OFL_EINVAL;
    }
    if (b->broken) {
        set_last_error("batch handle unusable after an earlier device error");
        return OFL_EDEVICE;
    }
    bool dev_err = false;
    const int rc = guarded(&dev_err, f);
    if (dev_err) {
        b->broken = true;
        for (ofl_grid *g : b->grids)
            g->broken = true;
    }
    return rc;
}

}  // namespace ofl
