// Many independent grids in one launch sequence.
//
// Every grid keeps its own arrays; the batch builds device tables (one view
// per grid plus work lists of tiles) and runs each nest of each iteration as
// ONE batched kernel over all grids. The whole iteration loop is captured
// once into a HIP graph and replayed, so a run is a single graph launch.
// Work lists are sorted largest grid first, so the longest tiles start early
// and the tail is made of small ones (longest-processing-time order).
// All three nests run on the GPU here (gene 111) with transfers hoisted out of
// the loop (paper Sec. 3.2.1): the read-only arrays and p move in before the
// loop, p moves back after it unless the grid's data region is open.
#include <algorithm>
#include <cmath>
#include <limits>
#include <memory>
#include <numeric>

#include "abi_util.hpp"
#include "batch.hpp"

namespace ofl {

namespace {

constexpr int kRowsPerWaveItem = 16;  // row tiles per wave in one residual/copy-back item

void free_dev(void *&p) {
    if (p) {
        (void)hipFree(p);
        p = nullptr;
    }
}

void drop_graph(ofl_batch *b) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    b->graph_iters = -1;
}

void free_tables(ofl_batch *b) {
    drop_graph(b);
    free_dev(b->d_views);
    free_dev(b->d_views_swapped);
    free_dev(b->d_fparts);
    free_dev(b->d_frange);
    free_dev(b->d_sitems);
    free_dev(b->d_ritems);
    free_dev(b->d_range);
    free_dev(b->d_partials);
    b->tables_ready = false;
}

template <class T>
void upload(void *&dst, const std::vector<T> &src, hipStream_t s) {
    free_dev(dst);
    const size_t bytes = std::max<size_t>(sizeof(T), src.size() * sizeof(T));
    hip_check(hipMalloc(&dst, bytes), "hipMalloc(batch table)");
    if (!src.empty())
        hip_check(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s),
                  "hipMemcpyAsync(batch table)");
}

}  // namespace

// Device view tables from the grids' current views: as held (even iterations)
// and with p and wrk2 exchanged (odd iterations of a swapping run).
void batch_upload_views(ofl_batch *b) {
    const size_t n = b->grids.size();
    std::vector<GridView> views(n), swapped(n);
    for (size_t g = 0; g < n; ++g) {
        views[g] = b->grids[g]->view;
        views[g].partials = static_cast<double *>(b->d_partials) + b->partial_base[g];
        views[g].nseg = b->nseg.empty() ? 0 : b->nseg[g];
        views[g].vec = b->gvec.empty() ? 0 : b->gvec[g];
        swapped[g] = views[g];
        std::swap(swapped[g].p, swapped[g].wrk2);
    }
    if (b->d_views && b->d_views_swapped) {
        // in place: a captured graph keeps reading these two buffers
        hip_check(hipMemcpyAsync(b->d_views, views.data(), n * sizeof(GridView), hipMemcpyHostToDevice, b->stream),
                  "hipMemcpyAsync(batch views)");
        hip_check(hipMemcpyAsync(b->d_views_swapped, swapped.data(), n * sizeof(GridView), hipMemcpyHostToDevice,
                                 b->stream),
                  "hipMemcpyAsync(batch views)");
    } else {
        upload(b->d_views, views, b->stream);
        upload(b->d_views_swapped, swapped, b->stream);
    }
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize(batch views)");
}

// Vector width for a grid of I points along i: the one whose wave tiles cover
// the interior with the fewest idle lanes; wider wins ties within 5%.
int batch_auto_vec(int I) {
    const int w = I - 2;
    int best = 4;
    double best_util = 0.0;
    for (int vec : {4, 2, 1}) {
        const int span = kWave * vec;
        const double util = static_cast<double>(w) / (span * ((w + span - 1) / span));
        if (util > best_util * 1.05) {
            best_util = util;
            best = vec;
        }
    }
    return best;
}

// Packed rows for a grid whose rows fill few of a wave's lanes. A wave then
// covers 64 * vec consecutive points of a plane across row ends, so its lanes
// idle only on the two boundary columns and the row padding, and a row no
// longer pays partial HBM granules at both of its ends. Worth it only when the
// rows are packed tightly (a small desc.row_align): with 128-byte rows the
// padding would be loaded and the lanes idle as before. Chosen when it keeps
// more lanes busy than one row per wave, and always when the compact rows do
// not start on 128-byte lines of p (a pitch that is not a multiple of 32
// elements): one row per wave would then split lines at both ends of every
// row load, while packed segments start on whole lines. Never for waves
// marching along j, nor for a grid whose coefficient rows have a pitch of
// their own (a segment runs across row ends, so every array must share p's
// rows and planes). Measured on 64 uneven grids with 4-element alignment:
// FP32 76.6 -> 77.7 GLUP/s (fused 99.1 -> 99.7), bfloat16-offset 111.9 ->
// 114.0 (fused 168.1 -> 170.3).
TileCfg batch_default_tile(int fmt, unsigned fusion) {
    TileCfg t;
    t.vec = 0;
    // One row per work-group: with the XCD bands of the item list it beat 4
    // rows in all four forms (FP32 73.8 against 73.2 GLUP/s, fused 94.0
    // against 93.2; bfloat16-offset 110.1 against 109.7, fused 163.3 against
    // 163.0).
    t.rows = 1;
    // 2-plane chunks for FP32 coefficients (77.8 against 76.1 GLUP/s, fused
    // 97.3 against 96.1), 4 for bfloat16 ones (113.3 against 112.3, fused
    // 166.0 against 160.2).
    t.kchunk = fmt == OFL_COEF_F32 ? 2 : 4;
    // Non-temporal stores as well: measured on 64 uneven grids they add 6% to
    // the plain batch and 7-18% to the fused one. (Ordinary stores in the
    // copy-back alone make it 1.6x faster, but the next sweep then writes the
    // dirty lines of p back and loses as much.)
    t.flags = OFL_TILE_NT_LOADS | OFL_TILE_NT_STORES;
    t.occupancy = 0;
    // The unfused bfloat16 batch: 4 points per lane in every grid and 2 rows
    // per work-group, the batch GA's pick, 114.5-114.6 against 113.5-113.6
    // GLUP/s on 64 uneven grids (fused, the GA's pick is within noise of the
    // tile above).
    if (fmt != OFL_COEF_F32 && fusion == 0) {
        t.vec = 4;
        t.rows = 2;
    }
    return t;
}

bool batch_packed(const Layout &L, const TileCfg &t, int *vec, int *nseg) {
    const int I = L.I, J = L.J, pitch = L.pitch;
    if ((t.flags & OFL_TILE_MARCH_J) || L.cpitch != pitch || L.cplane != L.plane)
        return false;
    // The packed kernels count a plane's points in 32-bit ints.
    if (static_cast<long long>(J) * pitch > 0x7fffffffLL - 4096)
        return false;
    const int vrow = t.vec > 0 ? t.vec : batch_auto_vec(I);
    const int vpk = t.vec > 0 ? t.vec : 4;
    if (pitch % vpk != 0)
        return false;
    const int span_row = kWave * vrow, span_pk = kWave * vpk;
    const long long segs = packed_nseg(J, pitch, vpk);
    const double util_row = static_cast<double>(I - 2) / (static_cast<double>(span_row) * itiles(I, vrow));
    const double util_pk = static_cast<double>(I - 2) * (J - 2) / (static_cast<double>(segs) * span_pk);
    const bool split_lines = pitch % kPitchAlign != 0;  // rows of p off 128-byte lines
    if ((!split_lines && util_pk <= util_row * 1.02) || segs > 0x7fffffffLL / 4)
        return false;
    *vec = vpk;
    *nseg = static_cast<int>(segs);
    return true;
}

namespace {

// Item w of a batched launch runs on XCD w % 8 (one work-group per item, or a
// multiple of 8 work-groups walking the list). Within one grid's items, every
// window of 8*q consecutive items (q = a k-chunk's items / 8, at least 1) is
// transposed so that each XCD receives q consecutive items: rows that share
// halo rows of p then meet in one L2 instead of being fetched by two XCDs. A
// grid's items stay a contiguous range of the list (its fused-residual slots
// depend on that); a tail shorter than a window keeps its order. Measured on
// 64 uneven grids with one row per work-group: FP32 72.6 -> 73.8 GLUP/s (fused
// 92.2 -> 94.0), bfloat16-offset 108.2 -> 110.1 (fused 159.2 -> 163.3).
void xcd_bands(std::vector<SweepItem> &items, size_t first, int per_chunk) {
    const size_t q = static_cast<size_t>(std::max(1, per_chunk / 8));
    const size_t window = 8 * q;
    std::vector<SweepItem> tmp(window);
    for (size_t base = first; base + window <= items.size(); base += window) {
        std::copy(items.begin() + static_cast<std::ptrdiff_t>(base),
                  items.begin() + static_cast<std::ptrdiff_t>(base + window), tmp.begin());
        for (size_t o = 0; o < window; ++o)
            items[base + (o % q) * 8 + o / q] = tmp[o];
    }
}

}  // namespace

void batch_build_tables(ofl_batch *b) {
    if (b->tables_ready)
        return;
    free_tables(b);
    const int n = static_cast<int>(b->grids.size());
    for (ofl_grid *g : b->grids)
        grid_ensure_device(g);
    // Largest grid first.
    std::vector<int> order(static_cast<size_t>(n));
    std::iota(order.begin(), order.end(), 0);
    auto interior = [&](int g) {
        const ofl_grid *q = b->grids[static_cast<size_t>(g)];
        return static_cast<long long>(q->I - 2) * (q->J - 2) * (q->K - 2);
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return interior(x) > interior(y); });

    // One item list per nest for every grid, largest grid first. With
    // tile.vec == 0 each grid gets the width that leaves the fewest idle lanes
    // on its interior rows, recorded in its view: one launch then runs items
    // of every width, each at its grid's own (no launch per width, so the
    // small grids fill the tail of the large ones instead of running after it).
    std::vector<SweepItem> sitems;
    std::vector<RowItem> ritems;
    std::vector<int> range(static_cast<size_t>(n) + 1, 0);
    std::vector<int> count(static_cast<size_t>(n), 0);
    const int rows_per_item = kRowsPerWaveItem * (kResidualThreads / kWave);
    b->nseg.assign(static_cast<size_t>(n), 0);
    b->gvec.assign(static_cast<size_t>(n), 0);
    for (int g : order) {
        const ofl_grid *q = b->grids[static_cast<size_t>(g)];
        TileCfg t = b->tile;
        int pvec = 0, nseg = 0;
        const bool packed = batch_packed(q->lay, b->tile, &pvec, &nseg);
        t.vec = packed ? pvec : (b->tile.vec > 0 ? b->tile.vec : batch_auto_vec(q->I));
        b->gvec[static_cast<size_t>(g)] = t.vec;
        int nti, nfb, nmc;
        if (packed) {
            // one "line" per segment; the kernels find the segment from fblock
            nti = 1;
            nfb = (nseg + t.rows - 1) / t.rows;
            nmc = (q->K - 2 + t.kchunk - 1) / t.kchunk;
            b->nseg[static_cast<size_t>(g)] = nseg;
        } else {
            sweep_shape(q->I, q->J, q->K, t, &nti, &nfb, &nmc);
        }
        const size_t first_item = sitems.size();
        for (int mc = 0; mc < nmc; ++mc)
            for (int fb = 0; fb < nfb; ++fb)
                for (int it = 0; it < nti; ++it)
                    sitems.push_back({g, it, fb, mc});
        if (!(b->tile.flags & OFL_TILE_XCD_REMAP))
            xcd_bands(sitems, first_item, nti * nfb);
        const long long nrt_l = packed ? static_cast<long long>(nseg) * (q->K - 2)
                                       : static_cast<long long>(nti) * (q->J - 2) * (q->K - 2);
        if (nrt_l > 0x7fffffffLL)
            fail(OFL_EINVAL, "a batched grid has too many row tiles");
        const int nrt = static_cast<int>(nrt_l);
        int slot = 0;
        for (int first = 0; first < nrt; first += rows_per_item) {
            ritems.push_back({g, first, std::min(rows_per_item, nrt - first), slot});
            ++slot;
        }
        count[static_cast<size_t>(g)] = slot;
    }
    if (sitems.size() > 0x7fffffffULL / static_cast<size_t>(std::max(1, b->tile.rows)) || ritems.size() > 0x7fffffffULL)
        fail(OFL_EINVAL, "the batch has too many work items");
    b->s_cnt = static_cast<int>(sitems.size());
    b->r_cnt = static_cast<int>(ritems.size());
    for (int g = 0; g < n; ++g)
        range[static_cast<size_t>(g) + 1] = range[static_cast<size_t>(g)] + count[static_cast<size_t>(g)];
    const hipStream_t s = b->stream;
    hip_check(hipMalloc(&b->d_partials, sizeof(double) * std::max(1, range[static_cast<size_t>(n)])),
              "hipMalloc(batch partials)");
    b->partial_base.assign(static_cast<size_t>(n), 0);
    for (int g = 0; g < n; ++g)
        b->partial_base[static_cast<size_t>(g)] = range[static_cast<size_t>(g)];
    batch_upload_views(b);
    // fused residual: grid g owns the partial slots of its sweep items (rows
    // slots per item), which are contiguous in the concatenated list; the
    // table holds [first slot, end slot) for every grid.
    std::vector<long long> frange(2 * static_cast<size_t>(n), 0);
    for (size_t w = sitems.size(); w-- > 0;)
        frange[2 * static_cast<size_t>(sitems[w].grid)] = static_cast<long long>(w) * b->tile.rows;
    for (size_t w = 0; w < sitems.size(); ++w)
        frange[2 * static_cast<size_t>(sitems[w].grid) + 1] = static_cast<long long>(w + 1) * b->tile.rows;
    // two buffers (even and odd iterations), each one partial per sweep wave
    b->fparts_len = static_cast<long long>(sitems.size()) * b->tile.rows;
    hip_check(hipMalloc(&b->d_fparts, sizeof(double) * std::max<size_t>(1, 2 * static_cast<size_t>(b->fparts_len))),
              "hipMalloc(batch fused partials)");
    upload(b->d_frange, frange, s);
    upload(b->d_sitems, sitems, s);
    upload(b->d_ritems, ritems, s);
    upload(b->d_range, range, s);
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize(batch tables)");
    b->tables_ready = true;
}

namespace {

}  // namespace

// A batch tile may leave the vector width to the batch (vec = 0).
bool batch_auto_vec_tile(const ofl_tile &t) {
    ofl_tile u = t;
    if (u.vec != 0)
        return false;
    u.vec = 4;
    return tile_valid(u, nullptr);
}

namespace {

int blocks_for(const ofl_batch *b, int nitems) {
    if (b->tile.occupancy <= 0)
        return std::max(1, nitems);
    return std::max(1, std::min(nitems, b->tile.occupancy * b->cu_count));
}

}  // namespace

// Enqueue iters x (S, R, finalize, C) for every grid on the batch stream:
// per nest one batched launch per vector-width class that has work. With
// OFL_FUSE_RESIDUAL the sweep emits the residual partials (then one finalize
// per grid); with OFL_FUSE_COPYBACK_SWAP there is no copy-back and odd
// iterations read the view table with p and wrk2 exchanged.
void batch_enqueue(ofl_batch *b, int iters, float omega) {
    const auto *views_even = static_cast<const GridView *>(b->d_views);
    const auto *views_odd = static_cast<const GridView *>(b->d_views_swapped);
    const auto *sitems = static_cast<const SweepItem *>(b->d_sitems);
    const auto *ritems = static_cast<const RowItem *>(b->d_ritems);
    const auto *range = static_cast<const int *>(b->d_range);
    auto *fparts = static_cast<double *>(b->d_fparts);
    const auto *frange = static_cast<const long long *>(b->d_frange);
    const bool fuse_r = (b->fusion & OFL_FUSE_RESIDUAL) != 0;
    const bool swap = (b->fusion & OFL_FUSE_COPYBACK_SWAP) != 0;
    const int n = static_cast<int>(b->grids.size());
    // tile.vec 0: every item runs at its grid's own width (views[].vec)
    const int vec = b->tile.vec;
    for (int it = 0; it < iters; ++it) {
        const GridView *views = (swap && (it & 1)) ? views_odd : views_even;
        // fused residual: iteration it writes partial buffer it % 2, and the
        // first work-groups of its sweep sum the previous iteration's buffer
        // into each grid's gosa; the last iteration's is summed after the loop
        double *cur = fuse_r ? fparts + (it & 1) * b->fparts_len : nullptr;
        PrevParts prev;
        if (fuse_r && it > 0) {
            prev.parts = fparts + ((it - 1) & 1) * b->fparts_len;
            prev.range = frange;
            prev.ngrids = n;
        }
        if (b->s_cnt > 0)
            launch_batch_sweep(views, sitems, b->s_cnt, b->tile, b->fmt != OFL_COEF_F32, omega,
                               blocks_for(b, b->s_cnt), b->stream, cur, prev);
        if (fuse_r) {
            if (it == iters - 1)
                launch_batch_fold_finalize(views, cur, frange, n, omega, kWave * b->tile.rows, b->stream);
        } else {
            if (b->r_cnt > 0)
                launch_batch_residual(views, ritems, b->r_cnt, vec, b->sum_mode, b->tile.flags,
                                      blocks_for(b, b->r_cnt), b->stream);
            launch_batch_finalize(views, range, n, omega, b->stream);
        }
        if (!swap && b->r_cnt > 0)
            launch_batch_copyback(views, ritems, b->r_cnt, vec, b->tile.flags, blocks_for(b, b->r_cnt), b->stream,
                                  true);
    }
}

void batch_prepare(ofl_batch *b) {
    TraceRange range("ofl:batch prepare");
    // Hoisted transfers before the loop: every grid's inputs to the device.
    for (ofl_grid *g : b->grids) {
        grid_ensure_device(g);
        std::vector<Xfer> xs;
        plan_enter(OFL_MASK_ALL_GPU, g->valid, xs);
        grid_exec(g, xs);
        // wrk2 carries p's boundary: needed by the buffer exchange, and lets
        // the copy-back write whole rows
        grid_sync_wrk2_boundary(g);
        grid_sync(g);
    }
    batch_build_tables(b);
}

void batch_launch(ofl_batch *b, int iters, float omega) {
    const bool reuse = b->exec && b->graph_iters == iters && b->graph_omega == omega && b->graph_fusion == b->fusion;
    if (!reuse) {
        drop_graph(b);
        hipGraph_t graph = nullptr;
        hip_check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
            batch_enqueue(b, iters, omega);
        } catch (...) {
            (void)hipStreamEndCapture(b->stream, &graph);
            if (graph)
                (void)hipGraphDestroy(graph);
            throw;
        }
        hip_check(hipStreamEndCapture(b->stream, &graph), "hipStreamEndCapture");
        const hipError_t e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        hip_check(e, "hipGraphInstantiate");
        b->graph_iters = iters;
        b->graph_omega = omega;
        b->graph_fusion = b->fusion;
    }
    TraceRange range("ofl:batch graph of iterations");
    hip_check(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
}

// State after a batched run: p and wrk2 hold their newest values on the device.
void batch_mark_done(ofl_batch *b, int iters) {
    for (ofl_grid *g : b->grids) {
        g->valid.dev[OFL_ARR_P] = 1;
        g->valid.host[OFL_ARR_P] = 0;
        g->valid.dev[OFL_ARR_WRK2] = 1;
        g->valid.host[OFL_ARR_WRK2] = 0;
        g->gosa_on_dev = true;
        for (int nest = 0; nest < 3; ++nest)
            g->stats.gpu_nests[nest] += static_cast<uint64_t>(iters);
    }
}

// After a swapping run of odd length every grid's p lives in its former
// wrk2 buffer: record the exchange and refresh both view tables in place.
void batch_after_run(ofl_batch *b, int iters) {
    if ((b->fusion & OFL_FUSE_COPYBACK_SWAP) && (iters & 1)) {
        for (ofl_grid *g : b->grids)
            grid_swap_p_wrk2(g);
        batch_upload_views(b);
    }
}

void batch_finish(ofl_batch *b, int iters, double *gosa_out) {
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize(batch)");
    batch_after_run(b, iters);
    batch_mark_done(b, iters);
    for (size_t t = 0; t < b->grids.size(); ++t) {
        ofl_grid *g = b->grids[t];
        if (!g->in_region) {
            std::vector<Xfer> xs;
            plan_sync_host(iters, g->valid, xs);
            grid_exec(g, xs);
        }
        hip_check(hipMemcpyAsync(&g->gosa_host, g->view.gosa, sizeof(double), hipMemcpyDeviceToHost, g->stream),
                  "hipMemcpyAsync(gosa)");
        g->gosa_on_dev = false;
        g->pending = true;
        grid_sync(g);
        if (gosa_out)
            gosa_out[t] = g->gosa_host;
    }
}

void batch_destroy_impl(ofl_batch *b) {
    if (!b)
        return;
    (void)hipSetDevice(b->device);
    if (b->stream)
        (void)hipStreamSynchronize(b->stream);
    free_tables(b);
    if (b->stream)
        (void)hipStreamDestroy(b->stream);
    for (ofl_grid *g : b->grids)
        g->batch_refs -= 1;
    delete b;
}

}  // namespace ofl

using namespace ofl;

extern "C" {

int ofl_batch_create(ofl_grid *const *grids, int n, const ofl_tile *tile, ofl_batch **out) {
    ofl_batch *made = nullptr;
    const int rc = guarded(nullptr, [&] {
        if (!grids || !out || n < 1)
            fail(OFL_EINVAL, "grids, out and n >= 1 are required");
        std::string why;
        if (tile && !(tile_valid(*tile, &why) || batch_auto_vec_tile(*tile)))
            fail(OFL_EINVAL, why);
        if (tile && tile->vec == 8)
            fail(OFL_ENOTSUP, "batched sweeps run 1, 2 or 4 points per lane (tile.vec 8 is for single grids)");
        for (int t = 0; t < n; ++t) {
            if (!grids[t])
                fail(OFL_EINVAL, "a grid handle is NULL");
            if (grids[t]->broken)
                fail(OFL_EDEVICE, "a grid handle is unusable after a device error");
            if (grids[t]->fmt != grids[0]->fmt || grids[t]->sum_mode != grids[0]->sum_mode)
                fail(OFL_EINVAL, "all grids of a batch need one coefficient format and sum mode");
            for (int u = 0; u < t; ++u)
                if (grids[u] == grids[t])
                    fail(OFL_EINVAL, "a grid appears twice in the batch");
            if (grids[t]->fusion != 0)
                fail(OFL_ESTATE, "a grid with fusion enabled cannot join a batch (ofl_set_fusion(g, 0) first)");
        }
        std::unique_ptr<ofl_batch> b(new ofl_batch);
        b->grids.assign(grids, grids + n);
        b->fmt = grids[0]->fmt;
        b->sum_mode = grids[0]->sum_mode;
        if (tile) {
            b->tile = to_cfg(*tile);
            b->tile_chosen = true;
        } else {
            b->tile = batch_default_tile(b->fmt, 0);
        }
        for (ofl_grid *g : b->grids)
            grid_ensure_device(g);
        b->device = grids[0]->device;
        for (ofl_grid *g : b->grids)
            if (g->device != b->device)
                fail(OFL_EINVAL, "all grids of a batch must live on one device");
        hip_check(hipSetDevice(b->device), "hipSetDevice");
        hip_check(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate(batch)");
        try {
            b->cu_count = device_cu_count(b->device);
        } catch (...) {
            (void)hipStreamDestroy(b->stream);
            throw;
        }
        for (ofl_grid *g : b->grids)
            g->batch_refs += 1;
        made = b.release();
    });
    if (rc == OFL_OK)
        *out = made;
    return rc;
}

void ofl_batch_destroy(ofl_batch *b) { batch_destroy_impl(b); }

int ofl_batch_set_tile(ofl_batch *b, const ofl_tile *tile) {
    return batch_call(b, [&] {
        if (!b || !tile)
            fail(OFL_EINVAL, "NULL argument");
        std::string why;
        if (!tile_valid(*tile, &why) && !batch_auto_vec_tile(*tile))
            fail(OFL_EINVAL, why);
        if (tile->vec == 8)
            fail(OFL_ENOTSUP, "batched sweeps run 1, 2 or 4 points per lane (tile.vec 8 is for single grids)");
        const TileCfg c = to_cfg(*tile);
        if (c.vec != b->tile.vec || c.rows != b->tile.rows || c.kchunk != b->tile.kchunk ||
            c.flags != b->tile.flags || c.occupancy != b->tile.occupancy) {
            hip_check(hipSetDevice(b->device), "hipSetDevice");
            hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
            free_tables(b);
            b->tile = c;
        }
        b->tile_chosen = true;
    });
}

int ofl_batch_set_fusion(ofl_batch *b, unsigned flags) {
    return batch_call(b, [&] {
        if (!b)
            fail(OFL_EINVAL, "NULL batch handle");
        if (flags & ~static_cast<unsigned>(OFL_FUSE_RESIDUAL | OFL_FUSE_COPYBACK_SWAP))
            fail(OFL_EINVAL, "unknown fusion bits");
        if ((flags & OFL_FUSE_RESIDUAL) && b->sum_mode != OFL_SUM_F64)
            fail(OFL_ENOTSUP, "the fused residual sums in FP64 only; this batch asks for compensated FP32");
        if (flags != b->fusion) {
            hip_check(hipSetDevice(b->device), "hipSetDevice");
            hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
            drop_graph(b);
            b->fusion = flags;
            if (!b->tile_chosen) {
                const TileCfg t = batch_default_tile(b->fmt, flags);
                if (t.vec != b->tile.vec || t.rows != b->tile.rows || t.kchunk != b->tile.kchunk ||
                    t.flags != b->tile.flags || t.occupancy != b->tile.occupancy) {
                    free_tables(b);
                    b->tile = t;
                }
            }
        }
    });
}

int ofl_batch_get_tile(const ofl_batch *b, ofl_tile *tile) {
    return guarded(nullptr, [&] {
        if (!b || !tile)
            fail(OFL_EINVAL, "NULL argument");
        *tile = to_tile(b->tile);
    });
}

int ofl_batch_run(ofl_batch *b, int iters, float omega, double *gosa_out) {
    return batch_call(b, [&] {
        if (!b)
            fail(OFL_EINVAL, "NULL batch handle");
        if (iters < 0)
            fail(OFL_EINVAL, "iters must be >= 0");
        if (!std::isfinite(omega) || omega == 0.f)
            fail(OFL_EINVAL, "omega must be finite and non-zero");
        for (ofl_grid *g : b->grids)
            if (g->broken)
                fail(OFL_EDEVICE, "a grid of the batch is unusable after a device error");
        if (iters == 0) {
            if (gosa_out)
                for (size_t t = 0; t < b->grids.size(); ++t)
                    gosa_out[t] = std::numeric_limits<double>::quiet_NaN();
            return;
        }
        hip_check(hipSetDevice(b->device), "hipSetDevice");
        batch_prepare(b);
        batch_launch(b, iters, omega);
        batch_finish(b, iters, gosa_out);
    });
}

}  // extern "C"
