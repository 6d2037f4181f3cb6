// Grid handle, transfer execution, the iteration driver and the grid part of
// the C interface.
//
// The iteration driver is the offloaded program's outer loop (paper Sec.
// 3.2.1): for every iteration it runs the sweep, residual and copy-back nests,
// each on the side its gene bit names, and before/after each nest issues the
// transfers the planner derives from the variable reference relations (Sec.
// 4.2.2).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <utility>
#include <cstring>
#include <limits>
#include <memory>

#include "abi_util.hpp"
#include "cpu_nests.hpp"
#include "grid.hpp"

namespace ofl {

namespace {

thread_local std::string t_last_error;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool row_align_valid(int a) { return a == 0 || a == 4 || a == 8 || a == 16 || a == 32; }

}  // namespace

void set_last_error(const std::string &msg) { t_last_error = msg; }

void fail(int code, const std::string &msg) { throw Error(code, msg); }

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess)
        throw Error(OFL_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

Layout make_layout(int I, int J, int K, int coef_format, int row_align) {
    Layout L;
    L.I = I;
    L.J = J;
    L.K = K;
    // By default every row starts on a 128-byte boundary: 32 elements of p and
    // wrk2, and 32 FP32 or 64 bfloat16 elements of the coefficient arrays. (A
    // 576-byte bfloat16 row would start every other row mid-line, and a wave's
    // 512-byte read would then touch five cache lines instead of four.) The
    // coefficient rows stop before i = I-1, a boundary column no nest reads, so
    // a row of 2^n + 1 points stores 2^n coefficients and the coefficient
    // streams run without gaps (the sweep streams gapped rows of 257 points
    // about 2-3% slower). A smaller row alignment packs short rows tighter and
    // keeps one layout for all arrays (packed batch rows run across row ends);
    // it stays a multiple of 4 elements, so every vector load of up to 4
    // elements starts on its own size.
    L.coef_elem = coef_format == OFL_COEF_F32 ? 4 : 2;
    if (row_align > 0) {
        L.pitch = round_up(I, row_align);
        L.plane = align_up(static_cast<size_t>(L.pitch) * J, static_cast<size_t>(kSegAlign));
        L.cpitch = L.pitch;
        L.crow = I;
        L.cplane = L.plane;
    } else {
        L.pitch = round_up(I, kPitchAlign);
        L.plane = static_cast<size_t>(L.pitch) * J;
        L.cpitch = round_up(I - 1, static_cast<int>(kPitchAlign * 4 / L.coef_elem));
        L.crow = std::min(I, L.cpitch);
        L.cplane = static_cast<size_t>(L.cpitch) * J;
    }
    L.elems = L.plane * K;
    L.celems = L.cplane * K;
    size_t off = 0;
    auto place = [&](size_t n, size_t eb) {
        off = align_up(off + kGuard * eb, 256);
        const size_t at = off;
        off += (n + kGuard) * eb;
        return at;
    };
    for (int a = 0; a < kNCoef; ++a)
        L.off[a] = place(L.celems, L.coef_elem);
    L.off[OFL_ARR_P] = place(L.elems, 4);
    L.off[OFL_ARR_WRK2] = place(L.elems, 4);
    L.staging_off = align_up(off, 256);
    off = L.staging_off + static_cast<size_t>(I) * J * K * 4;
    L.partials_off = align_up(off, 256);
    off = L.partials_off + sizeof(double) * kResidualBlocks;
    L.gosa_off = align_up(off, 256);
    off = L.gosa_off + 256;
    L.total = align_up(off, 4096);
    return L;
}

bool tile_valid(const ofl_tile &t, std::string *why) {
    auto bad = [&](const char *m) {
        if (why)
            *why = m;
        return false;
    };
    if (t.vec != 1 && t.vec != 2 && t.vec != 4 && t.vec != 8)
        return bad("tile.vec must be 1, 2, 4 or 8");
    if (t.vec == 8 && (t.flags & OFL_TILE_MARCH_J))
        return bad("tile.vec 8 (two rows per wave) marches along k only: no OFL_TILE_MARCH_J");
    if (t.rows < 1 || t.rows > 8)
        return bad("tile.rows must be in 1..8");
    if (t.kchunk < 1 || t.kchunk > 1024)
        return bad("tile.kchunk must be in 1..1024");
    if (t.flags < 0 || t.flags > 31)
        return bad("tile.flags has unknown bits");
    if (t.occupancy < 0 || t.occupancy > 16)
        return bad("tile.occupancy must be in 0..16");
    return true;
}

TileCfg to_cfg(const ofl_tile &t) {
    TileCfg c;
    c.vec = t.vec;
    c.rows = t.rows;
    c.kchunk = t.kchunk;
    c.flags = t.flags;
    c.occupancy = t.occupancy;
    return c;
}

ofl_tile to_tile(const TileCfg &c) {
    ofl_tile t;
    t.vec = c.vec;
    t.rows = c.rows;
    t.kchunk = c.kchunk;
    t.flags = c.flags;
    t.occupancy = c.occupancy;
    return t;
}

TileCfg default_tile(int I, int fmt, unsigned fusion) {
    TileCfg t;
    const int interior = I - 2;
    t.vec = interior > 128 ? 4 : (interior > 64 ? 2 : 1);
    t.rows = 4;
    // 2-plane chunks: twice the work-groups of 4-plane ones keep more loads
    // in flight. Non-temporal stores of wrk2 for FP32 coefficients, and for
    // bfloat16 ones when the copy-back is a buffer exchange (the sweep's
    // output is then next read a whole sweep later). Measured at 257x257x513,
    // steps of 100 iterations, GLUP/s against 4-plane chunks with NT loads
    // only: FP32 83.6 / 82.6, fused 103.6 / 99.4; bfloat16-offset 123.1 /
    // 120.8 (NT stores there: 121.3), fused with NT stores 169.3 against 160.6.
    t.kchunk = 2;
    t.flags = OFL_TILE_NT_LOADS;
    if (fmt == OFL_COEF_F32 || (fusion & OFL_FUSE_COPYBACK_SWAP) != 0)
        t.flags |= OFL_TILE_NT_STORES;
    // The FP32 sweep at 4 points per lane streams its 14 arrays fastest with
    // 3 waves per SIMD, though its registers would admit 4: at most 3 resident
    // work-groups per CU. Unless the residual is fused into it, it also loads
    // each step's coefficients one step ahead (its registers then admit only
    // 3 waves anyway). Measured at 257x257x513 on one box, us per sweep: 317.2
    // uncapped, 313.8-314.0 capped, 310.1-311.3 capped with the early loads;
    // fused 316.6-316.9, 314.0 capped, 331.1 with the early loads. Capping
    // slows the other forms: bfloat16-offset 190.4 against 183.3 us there,
    // FP32 at 2 points per lane (129x129x257) 48.8 against 46.8.
    if (fmt == OFL_COEF_F32 && t.vec == 4) {
        t.occupancy = 3;
        if ((fusion & OFL_FUSE_RESIDUAL) == 0)
            t.flags |= OFL_TILE_PREFETCH;
    } else {
        t.occupancy = 0;
    }
    return t;
}

void sweep_shape(int I, int J, int K, const TileCfg &t, int *nti, int *nfb, int *nmc) {
    const bool march_j = (t.flags & OFL_TILE_MARCH_J) != 0;
    *nti = itiles(I, t.vec);
    // lines per work-group: one per wave, or two rows per wave at 8 points per lane
    const int lines = t.rows * (t.vec == 8 ? 2 : 1);
    *nfb = ((march_j ? K : J) - 2 + lines - 1) / lines;
    *nmc = ((march_j ? J : K) - 2 + t.kchunk - 1) / t.kchunk;
}

long long sweep_waves(int I, int J, int K, const TileCfg &t) {
    int nti, nfb, nmc;
    sweep_shape(I, J, K, t, &nti, &nfb, &nmc);
    return static_cast<long long>(nti) * nfb * nmc * t.rows;
}

void *grid_array_ptr(ofl_grid *g, int a) { return g->block + g->lay.off[a]; }

void grid_ensure_device(ofl_grid *g) {
    if (g->dev_ready) {
        hip_check(hipSetDevice(g->device), "hipSetDevice");
        return;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        fail(OFL_EDEVICE, "a GPU nest was requested but no HIP device is available");
    int dev = g->want_device;
    if (dev < 0)
        hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev >= count)
        fail(OFL_EINVAL, "desc.device is not a valid HIP device ordinal");
    hip_check(hipSetDevice(dev), "hipSetDevice");
    const Layout lay = make_layout(g->I, g->J, g->K, g->fmt, g->row_align);
    if (g->arena && g->arena_bytes < lay.total)
        fail(OFL_ENOMEM, "dev_arena is smaller than ofl_grid_device_bytes()");
    // Take the block and the stream, and zero the block, before the grid
    // records any of it: a failure on the way releases what was taken and
    // leaves the grid without device state, as before the call.
    char *block = static_cast<char *>(g->arena);
    bool own_block = false;
    hipStream_t stream = static_cast<hipStream_t>(g->user_stream);
    bool own_stream = false;
    try {
        if (!block) {
            void *ptr = nullptr;
            const hipError_t e = hipMalloc(&ptr, lay.total);
            if (e != hipSuccess)
                fail(OFL_ENOMEM, std::string("hipMalloc of the grid's device block failed: ") + hipGetErrorString(e));
            block = static_cast<char *>(ptr);
            own_block = true;
        }
        if (!stream) {
            hip_check(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking), "hipStreamCreate");
            own_stream = true;
        }
        // Zero the whole block once (guards and padding included) so that every
        // value a wave may read past a row end is defined.
        launch_fill_zero(block, lay.total, stream);
    } catch (...) {
        if (own_stream)
            (void)hipStreamDestroy(stream);
        if (own_block)
            (void)hipFree(block);
        throw;
    }
    g->device = dev;
    g->lay = lay;
    g->block = block;
    g->own_block = own_block;
    g->stream = stream;
    g->own_stream = own_stream;
    GridView &v = g->view;
    v.p = reinterpret_cast<float *>(g->block + g->lay.off[OFL_ARR_P]);
    v.wrk2 = reinterpret_cast<float *>(g->block + g->lay.off[OFL_ARR_WRK2]);
    for (int a = 0; a < kNCoef; ++a) {
        v.coef[a] = g->block + g->lay.off[a];
        v.bias[a] = g->bias[a];
    }
    v.I = g->I;
    v.J = g->J;
    v.K = g->K;
    v.pitch = g->lay.pitch;
    v.cpitch = g->lay.cpitch;
    v.nseg = 0;
    v.vec = 0;
    v.plane = static_cast<long long>(g->lay.plane);
    v.cplane = static_cast<long long>(g->lay.cplane);
    v.partials = reinterpret_cast<double *>(g->block + g->lay.partials_off);
    v.gosa = reinterpret_cast<double *>(g->block + g->lay.gosa_off);
    g->dev_ready = true;
    g->pending = true;
}

namespace {

size_t array_elem_bytes(const ofl_grid *g, int a) { return (a < kNCoef && g->fmt != OFL_COEF_F32) ? 2 : 4; }

const void *host_src(const ofl_grid *g, int a) {
    if (a < kNCoef)
        return g->fmt == OFL_COEF_F32 ? static_cast<const void *>(g->coef[a])
                                       : static_cast<const void *>(g->enc[a].data());
    return a == OFL_ARR_P ? g->p : g->wrk2;
}

void harvest_events(ofl_grid *g) {
    for (size_t t = 0; t < g->ev_used; ++t) {
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, g->ev[2 * t], g->ev[2 * t + 1]), "hipEventElapsedTime");
        const int nest = g->ev_nest[t];
        g->stats.kernel_ms[nest] += ms;
        g->stats.timed_nests[nest] += 1;
    }
    g->ev_used = 0;
}

void prof_begin(ofl_grid *g, int nest) {
    g->prof_open = g->profiling && ((g->prof_nests >> nest) & 1u);
    if (!g->prof_open)
        return;
    if (g->ev.size() < 2 * (g->ev_used + 1)) {
        for (int t = 0; t < 2; ++t) {
            // Timing only (read after a stream synchronisation): no system-scope
            // fence, which would write back and invalidate the caches between
            // nests and slow the work being timed.
            hipEvent_t e;
            hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreateWithFlags");
            g->ev.push_back(e);
        }
        g->ev_nest.push_back(0);
    }
    g->ev_nest[g->ev_used] = nest;
    hip_check(hipEventRecord(g->ev[2 * g->ev_used], g->stream), "hipEventRecord");
}

void prof_end(ofl_grid *g) {
    if (!g->prof_open)
        return;
    hip_check(hipEventRecord(g->ev[2 * g->ev_used + 1], g->stream), "hipEventRecord");
    g->ev_used += 1;
    g->prof_open = false;
}

// fold: the residual's finalize step runs inside the copy-back kernel that
// follows it (both nests on the GPU as whole nests, hoisted transfers), which
// saves one launch per iteration.
// Marker-range names: nests by index, transfers by array and direction.
const char *const kNestRange[3] = {"ofl:gpu sweep", "ofl:gpu residual", "ofl:gpu copy-back"};
const char *const kCpuNestRange[3] = {"ofl:cpu sweep", "ofl:cpu residual", "ofl:cpu copy-back"};
const char *const kRegionRange[3] = {"ofl:gpu sweep regions", "ofl:gpu residual regions", "ofl:gpu copy-back regions"};
const char *const kXferRange[2][14] = {
    {"ofl:h2d a0", "ofl:h2d a1", "ofl:h2d a2", "ofl:h2d a3", "ofl:h2d b0", "ofl:h2d b1", "ofl:h2d b2", "ofl:h2d c0",
     "ofl:h2d c1", "ofl:h2d c2", "ofl:h2d bnd", "ofl:h2d wrk1", "ofl:h2d p", "ofl:h2d wrk2"},
    {"ofl:d2h a0", "ofl:d2h a1", "ofl:d2h a2", "ofl:d2h a3", "ofl:d2h b0", "ofl:d2h b1", "ofl:d2h b2", "ofl:d2h c0",
     "ofl:d2h c1", "ofl:d2h c2", "ofl:d2h bnd", "ofl:d2h wrk1", "ofl:d2h p", "ofl:d2h wrk2"}};

// Store kind of a single grid's copy-back. The sweep that follows reads every
// plane of p again; when p fits in the last-level cache (256 MB on MI355X) with
// room to spare, ordinary stores leave it there and that sweep reads it from
// the cache, so the copy-back then ignores OFL_TILE_NT_STORES. Measured with
// FP32 coefficients (whole steps, GLUP/s, non-temporal -> ordinary stores; p's
// pitched bytes): 21 MB 62.9 -> 62.0, 67 MB 77.2 -> 78.7, 76 MB 82.8 -> 83.3,
// 114 MB 84.1 -> 85.5, 144 MB 85.2 -> 86.0, 152 MB 84.8 -> 85.6, 213 MB 65.7 ->
// 67.7, 290 MB 68.7 -> 67.5, 490 MB 71.9 -> 70.7. (The 64-grid batch, whose p
// arrays come to 0.5 GB, keeps the tile's stores.)
int copyback_flags(const ofl_grid *g) {
    constexpr size_t kMin = size_t{48} << 20, kMax = size_t{224} << 20;
    const size_t p_bytes = g->lay.elems * sizeof(float);
    if (p_bytes >= kMin && p_bytes <= kMax)
        return g->tile.flags & ~OFL_TILE_NT_STORES;
    return g->tile.flags;
}

void gpu_nest(ofl_grid *g, int nest, float omega, bool fold) {
    TraceRange range(kNestRange[nest]);
    prof_begin(g, nest);
    if (nest == kS) {
        launch_sweep(g->view, g->tile, g->fmt != OFL_COEF_F32, omega, g->stream);
    } else if (nest == kR) {
        launch_residual(g->view, g->tile.vec, g->sum_mode, g->tile.flags, omega, g->stream, !fold);
        g->gosa_on_dev = true;
    } else {
        launch_copyback(g->view, g->tile.vec, copyback_flags(g), g->stream, g->wrk2_boundary_ok, fold, omega);
    }
    prof_end(g);
    g->stats.gpu_nests[nest] += 1;
    g->stats.gpu_regions[nest] += 1;
    g->pending = true;
}

void check_deadline(const ofl_grid *g) {
    if (g->deadline_ns == 0)
        return;
    const long long now = std::chrono::duration_cast<std::chrono::nanoseconds>(
                              std::chrono::steady_clock::now().time_since_epoch())
                              .count();
    if (now > g->deadline_ns)
        throw Timeout{};
}

// Interior planes [k0, k1) x rows [j0, j1) of a nest split into regions.
struct Region {
    int k0, k1, j0, j1;
};

// The same arrays seen as the sub-box of planes k0-1..k1 and rows j0-1..j1:
// its interior is the region, and the kernels run on it unchanged (they address
// rows by pitch and planes by plane, which stay those of the whole grid).
GridView region_view(const GridView &v, const Region &r, size_t coef_bytes) {
    GridView s = v;
    const long long off = static_cast<long long>(r.k0 - 1) * v.plane + static_cast<long long>(r.j0 - 1) * v.pitch;
    const long long coff = static_cast<long long>(r.k0 - 1) * v.cplane + static_cast<long long>(r.j0 - 1) * v.cpitch;
    s.p = v.p + off;
    s.wrk2 = v.wrk2 + off;
    for (int a = 0; a < kNCoef; ++a)
        s.coef[a] = static_cast<const char *>(v.coef[a]) + coff * static_cast<long long>(coef_bytes);
    s.J = r.j1 - r.j0 + 2;
    s.K = r.k1 - r.k0 + 2;
    return s;
}

// Rows [j0, j1) of planes [k0, k1) of array a between host and device, one
// pitched copy per plane (the host rows of a plane are contiguous).
void xfer_box(ofl_grid *g, int a, int dir, int k0, int k1, int j0, int j1) {
    const size_t eb = array_elem_bytes(g, a);
    const size_t row = static_cast<size_t>(g->I) * eb;
    const bool coef = a < kNCoef;
    const size_t pitch = static_cast<size_t>(coef ? g->lay.cpitch : g->lay.pitch);
    const size_t plane = coef ? g->lay.cplane : g->lay.plane;
    const size_t width = static_cast<size_t>(coef ? g->lay.crow : g->I) * eb;  // bytes kept of each host row
    char *dev = static_cast<char *>(grid_array_ptr(g, a));
    for (int k = k0; k < k1; ++k) {
        const size_t hoff = (static_cast<size_t>(k) * g->J + j0) * row;
        const size_t doff = (static_cast<size_t>(k) * plane + static_cast<size_t>(j0) * pitch) * eb;
        if (dir == 0) {
            const char *src = static_cast<const char *>(host_src(g, a)) + hoff;
            hip_check(
                hipMemcpy2DAsync(dev + doff, pitch * eb, src, row, width, j1 - j0, hipMemcpyHostToDevice, g->stream),
                "hipMemcpy2DAsync(host->device rows)");
        } else {
            char *dst = reinterpret_cast<char *>(a == OFL_ARR_P ? g->p : g->wrk2) + hoff;
            hip_check(hipMemcpy2DAsync(dst, row, dev + doff, pitch * eb, row, j1 - j0, hipMemcpyDeviceToHost, g->stream),
                      "hipMemcpy2DAsync(device->host rows)");
        }
    }
    const uint64_t bytes = static_cast<uint64_t>(k1 - k0) * static_cast<uint64_t>(j1 - j0) * row;
    if (dir == 0) {
        g->stats.h2d_count += 1;
        g->stats.h2d_bytes += bytes;
        if (a == OFL_ARR_P || a == OFL_ARR_WRK2)
            g->wrk2_boundary_ok = false;
    } else {
        g->stats.d2h_count += 1;
        g->stats.d2h_bytes += bytes;
    }
    g->pending = true;
}

// A GPU nest whose region opens below the k loop: the host runs the outer
// loop(s) and launches the nest's kernel once per plane (OFL_LEVEL_J) or per
// row (OFL_LEVEL_I). With per_iter, each region first copies in the rows of
// `ins` it reads and afterwards copies out the rows of `out` it wrote, and a
// residual region's sum comes home at once.
void gpu_nest_regions(ofl_grid *g, int nest, float omega, bool per_iter, const std::vector<int> &ins, int out) {
    TraceRange range(kRegionRange[nest]);
    const int lev = g->level[nest];
    const int nk = g->K - 2, nj = g->J - 2;
    const long long nreg = lev == OFL_LEVEL_J ? nk : static_cast<long long>(nk) * nj;
    const size_t cb = g->lay.coef_elem;
    if (nest == kR) {
        if (nreg > g->region_sums_cap) {
            grid_sync(g);
            if (g->region_sums)
                hip_check(hipFree(g->region_sums), "hipFree(region sums)");
            g->region_sums = nullptr;
            g->region_sums_cap = 0;
            void *ptr = nullptr;
            hip_check(hipMalloc(&ptr, sizeof(double) * static_cast<size_t>(nreg)), "hipMalloc(region sums)");
            g->region_sums = static_cast<double *>(ptr);
            g->region_sums_cap = nreg;
        }
        if (per_iter)
            g->region_host.assign(static_cast<size_t>(nreg), 0.0);
    }
    if (!per_iter)
        prof_begin(g, nest);
    const int row_trips = lev == OFL_LEVEL_J ? 1 : nj;  // host trips of the j loop inside each k trip
    long long idx = 0;
    for (int k = 1; k <= nk; ++k) {
        for (int t = 0; t < row_trips; ++t, ++idx) {
            check_deadline(g);
            const Region r = lev == OFL_LEVEL_J ? Region{k, k + 1, 1, g->J - 1} : Region{k, k + 1, t + 1, t + 2};
            if (per_iter) {
                for (int a : ins) {
                    const bool halo = nest == kS && a == OFL_ARR_P;  // the stencil's p rows and planes
                    // whole planes at OFL_LEVEL_J (the boundary rows ride along), rows at OFL_LEVEL_I
                    const int j0 = lev == OFL_LEVEL_J ? 0 : (halo ? r.j0 - 1 : r.j0);
                    const int j1 = lev == OFL_LEVEL_J ? g->J : (halo ? r.j1 + 1 : r.j1);
                    xfer_box(g, a, 0, halo ? r.k0 - 1 : r.k0, halo ? r.k1 + 1 : r.k1, j0, j1);
                }
            }
            GridView v = region_view(g->view, r, cb);
            if (nest == kS) {
                launch_sweep(v, g->tile, g->fmt != OFL_COEF_F32, omega, g->stream);
            } else if (nest == kR) {
                v.gosa = g->region_sums + idx;
                launch_residual(v, g->tile.vec, g->sum_mode, g->tile.flags, 1.0f, g->stream);
                if (per_iter)
                    hip_check(hipMemcpyAsync(&g->region_host[static_cast<size_t>(idx)], v.gosa, sizeof(double),
                                             hipMemcpyDeviceToHost, g->stream),
                              "hipMemcpyAsync(region sum)");
            } else {
                launch_copyback(v, g->tile.vec, copyback_flags(g), g->stream);
            }
            g->stats.gpu_regions[nest] += 1;
            g->pending = true;
            if (per_iter && out >= 0)
                xfer_box(g, out, 1, r.k0, r.k1, lev == OFL_LEVEL_J ? 0 : r.j0, lev == OFL_LEVEL_J ? g->J : r.j1);
        }
    }
    if (nest == kR) {
        if (per_iter) {
            grid_sync(g);
            double sum = 0.0;
            for (double x : g->region_host)
                sum += x;
            const double w = static_cast<double>(omega);
            g->gosa_host = sum / (w * w);
            g->gosa_on_dev = false;
        } else {
            launch_finalize(g->region_sums, nreg, omega, g->view.gosa, g->stream, g->view.partials, kResidualBlocks);
            g->gosa_on_dev = true;
        }
    }
    if (!per_iter)
        prof_end(g);
    g->stats.gpu_nests[nest] += 1;
}

void cpu_nest(ofl_grid *g, int nest, float omega) {
    TraceRange range(kCpuNestRange[nest]);
    if (g->pending)
        grid_sync(g);
    if (nest == kS) {
        if (g->fmt == OFL_COEF_F32) {
            cpu_sweep_f32(g->I, g->J, g->K, g->coef, g->p, g->wrk2, omega);
        } else {
            const uint16_t *enc[kNCoef];
            for (int a = 0; a < kNCoef; ++a)
                enc[a] = g->enc[a].data();
            cpu_sweep_bf16(g->I, g->J, g->K, enc, g->bias, g->p, g->wrk2, omega);
        }
    } else if (nest == kR) {
        g->gosa_host = cpu_residual(g->I, g->J, g->K, g->p, g->wrk2, omega);
        g->gosa_on_dev = false;
    } else {
        cpu_copyback(g->I, g->J, g->K, g->wrk2, g->p);
    }
    g->stats.cpu_nests[nest] += 1;
}

}  // namespace

namespace {


// Fused iterations (gene 111, hoisted, fusion requested): the sweep also
// produces the residual's per-wave partials (OFL_FUSE_RESIDUAL), and the
// copy-back becomes a buffer exchange (OFL_FUSE_COPYBACK_SWAP), which is exact
// because wrk2's boundary was made equal to p's first and the sweep writes
// outside the interior only p's own values. The three nests still count as
// executed on the GPU.
//
// The partials are double-buffered: iteration it writes buffer it % 2, and
// the first work-group of its sweep sums buffer (it - 1) % 2, the previous
// iteration's, into gosa before its own march, so no iteration launches a
// reduction kernel of its own; the last iteration's is summed after the loop.
//
// static_parts != nullptr: the partials go there (at least twice
// sweep_waves() slots, checked by the caller) and nothing is allocated.
void run_fused(ofl_grid *g, int iters, float omega, double *static_parts = nullptr) {
    grid_ensure_device(g);
    std::vector<Xfer> xs;
    const bool fuse_r = (g->fusion & OFL_FUSE_RESIDUAL) != 0;
    const bool swap = (g->fusion & OFL_FUSE_COPYBACK_SWAP) != 0;
    const long long need = fuse_r ? sweep_waves(g->I, g->J, g->K, g->tile) : 0;
    double *parts = static_parts;
    if (fuse_r && !static_parts) {
        if (2 * need > g->fused_parts_cap) {
            grid_sync(g);
            if (g->fused_parts)
                hip_check(hipFree(g->fused_parts), "hipFree(fused partials)");
            g->fused_parts = nullptr;
            g->fused_parts_cap = 0;
            void *ptr = nullptr;
            hip_check(hipMalloc(&ptr, sizeof(double) * static_cast<size_t>(2 * need)), "hipMalloc(fused partials)");
            g->fused_parts = static_cast<double *>(ptr);
            g->fused_parts_cap = 2 * need;
        }
        parts = g->fused_parts;
    }
    for (int it = 0; it < iters; ++it) {
        TraceRange range("ofl:fused iteration");
        xs.clear();
        plan_before(it, kS, true, OFL_XFER_HOISTED, g->valid, xs);
        grid_exec(g, xs);
        if (swap)
            grid_sync_wrk2_boundary(g);
        double *cur = fuse_r ? parts + (it & 1) * need : nullptr;
        PrevParts prev;
        if (fuse_r && it > 0) {
            prev.parts = parts + ((it - 1) & 1) * need;
            prev.n = need;
        }
        prof_begin(g, kS);
        launch_sweep(g->view, g->tile, g->fmt != OFL_COEF_F32, omega, g->stream, cur, prev);
        prof_end(g);
        g->stats.gpu_nests[kS] += 1;
        xs.clear();
        plan_after(it, kS, true, OFL_XFER_HOISTED, g->valid, xs);
        if (fuse_r) {
            // this iteration's terms are in `cur`; the next sweep sums them
            if (it == iters - 1) {
                prof_begin(g, kR);
                launch_fold_finalize(cur, need, omega, g->view.gosa, kWave * g->tile.rows, g->stream);
                prof_end(g);
            }
        } else {
            prof_begin(g, kR);
            launch_residual(g->view, g->tile.vec, g->sum_mode, g->tile.flags, omega, g->stream);
            prof_end(g);
        }
        g->gosa_on_dev = true;
        g->stats.gpu_nests[kR] += 1;
        if (swap) {
            grid_swap_p_wrk2(g);
        } else {
            prof_begin(g, kC);
            launch_copyback(g->view, g->tile.vec, copyback_flags(g), g->stream, g->wrk2_boundary_ok);
            prof_end(g);
        }
        plan_after(it, kC, true, OFL_XFER_HOISTED, g->valid, xs);
        g->stats.gpu_nests[kC] += 1;
        g->pending = true;
    }
}

}  // namespace

// The outer loop of the offloaded program: iters x (S, R[, C]).
bool grid_whole_nests(const ofl_grid *g) {
    for (int n = 0; n < 3; ++n)
        if (((g->mask >> n) & 1u) && g->level[n] != OFL_LEVEL_K)
            return false;
    return true;
}

namespace {

// ---- steady-state iterations from captured HIP graphs
//
// With every nest on the GPU as one region, hoisted transfers, no fusion, no
// profiling events and no time limit, an iteration after the first is three
// kernel launches (sweep, residual + its finalize, copy-back) and nothing
// else: no transfer, no host work. Small grids are then bound by launch
// overhead, so those iterations are captured once into a graph of up to
// kGraphIters iterations and replayed. The capture records kernel launches
// only (no memset or copy nodes). A graph is reused while the grid's view,
// tile, omega and length are those it was captured with.
constexpr int kGraphIters = 256;

bool same_view(const GridView &a, const GridView &b) {
    for (int n = 0; n < kNCoef; ++n)
        if (a.coef[n] != b.coef[n] || a.bias[n] != b.bias[n])
            return false;
    return a.p == b.p && a.wrk2 == b.wrk2 && a.I == b.I && a.J == b.J && a.K == b.K && a.pitch == b.pitch &&
           a.cpitch == b.cpitch && a.nseg == b.nseg && a.plane == b.plane && a.cplane == b.cplane &&
           a.partials == b.partials && a.gosa == b.gosa;
}

bool same_tile(const TileCfg &a, const TileCfg &b) {
    return a.vec == b.vec && a.rows == b.rows && a.kchunk == b.kchunk && a.flags == b.flags &&
           a.occupancy == b.occupancy;
}

bool graph_eligible(const ofl_grid *g, int nests) {
    return nests == 3 && g->mask == OFL_MASK_ALL_GPU && g->mode == OFL_XFER_HOISTED && g->fusion == 0 &&
           !g->profiling && g->deadline_ns == 0 && grid_whole_nests(g);
}

void enqueue_iterations(ofl_grid *g, int iters, float omega) {
    for (int it = 0; it < iters; ++it) {
        launch_sweep(g->view, g->tile, g->fmt != OFL_COEF_F32, omega, g->stream);
        launch_residual(g->view, g->tile.vec, g->sum_mode, g->tile.flags, omega, g->stream, false);
        launch_copyback(g->view, g->tile.vec, copyback_flags(g), g->stream, g->wrk2_boundary_ok, true, omega);
    }
}

// A graph of `iters` steady-state iterations, cached; nullptr when the stream
// cannot be captured (for instance because the caller is capturing it).
hipGraphExec_t loop_graph(ofl_grid *g, int iters, float omega) {
    for (const auto &c : g->graphs)
        if (c.exec && c.iters == iters && c.omega == omega && c.whole_rows == g->wrk2_boundary_ok &&
            same_tile(c.tile, g->tile) && same_view(c.view, g->view))
            return c.exec;
    hipStreamCaptureStatus status = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(g->stream, &status) != hipSuccess || status != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return nullptr;
    }
    auto &slot = g->graphs[g->graph_next];
    g->graph_next ^= 1;
    if (slot.exec) {
        hip_check(hipGraphExecDestroy(slot.exec), "hipGraphExecDestroy");
        slot.exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    hip_check(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        enqueue_iterations(g, iters, omega);
    } catch (...) {
        (void)hipStreamEndCapture(g->stream, &graph);
        if (graph)
            (void)hipGraphDestroy(graph);
        throw;
    }
    hip_check(hipStreamEndCapture(g->stream, &graph), "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(e, "hipGraphInstantiate");
    slot.exec = exec;
    slot.view = g->view;
    slot.tile = g->tile;
    slot.omega = omega;
    slot.iters = iters;
    slot.whole_rows = g->wrk2_boundary_ok;
    return exec;
}

// Iterations [from, iters) from graphs, if the planner moves nothing in them:
// one iteration from the current state must plan no transfer and leave the
// state as it was (then every later one does the same). Returns the number of
// iterations run.
int run_graphed(ofl_grid *g, int from, int iters, float omega) {
    Validity v = g->valid;
    std::vector<Xfer> xs;
    for (int nest = 0; nest < 3; ++nest) {
        plan_before(from, nest, true, g->mode, v, xs);
        plan_after(from, nest, true, g->mode, v, xs);
    }
    if (!xs.empty() || std::memcmp(&v, &g->valid, sizeof v) != 0)
        return 0;
    int done = 0;
    while (from + done < iters) {
        const int n = std::min(iters - from - done, kGraphIters);
        hipGraphExec_t exec = loop_graph(g, n, omega);
        if (!exec)
            break;
        {
            TraceRange range("ofl:graph of iterations");
            hip_check(hipGraphLaunch(exec, g->stream), "hipGraphLaunch");
        }
        done += n;
    }
    for (int nest = 0; nest < 3; ++nest) {
        g->stats.gpu_nests[nest] += static_cast<uint64_t>(done);
        g->stats.gpu_regions[nest] += static_cast<uint64_t>(done);
    }
    if (done > 0) {
        g->gosa_on_dev = true;
        g->pending = true;
    }
    return done;
}

}  // namespace

void grid_drop_graphs(ofl_grid *g) {
    for (auto &c : g->graphs)
        if (c.exec) {
            (void)hipGraphExecDestroy(c.exec);
            c.exec = nullptr;
        }
}

void grid_run_loop(ofl_grid *g, int iters, float omega, int nests) {
    if (nests == 3 && g->fusion != 0 && g->mask == OFL_MASK_ALL_GPU && g->mode == OFL_XFER_HOISTED &&
        g->batch_refs == 0 && grid_whole_nests(g)) {
        run_fused(g, iters, omega);
        return;
    }
    // Every nest on the GPU as one region with hoisted transfers: after the
    // first iteration's uploads, give the device wrk2 p's boundary once, so the
    // copy-back writes whole rows from then on.
    const bool resident = nests == 3 && g->mask == OFL_MASK_ALL_GPU && g->mode == OFL_XFER_HOISTED &&
                          g->fusion == 0 && grid_whole_nests(g);
    const bool graphed = graph_eligible(g, nests) && iters > 1;
    // The residual's finalize step runs inside the copy-back kernel when both
    // nests run on the GPU as whole nests with hoisted transfers (nothing reads
    // gosa between them), and not under a search's time limit, which may stop
    // a run between the two.
    const bool fold = nests == 3 && (g->mask & 6u) == 6u && g->mode == OFL_XFER_HOISTED &&
                      g->level[kR] == OFL_LEVEL_K && g->level[kC] == OFL_LEVEL_K && g->deadline_ns == 0;
    std::vector<Xfer> xs;
    std::vector<int> ins;
    for (int it = 0; it < iters; ++it) {
        if (resident && it == 1)
            grid_sync_wrk2_boundary(g);
        if (graphed && it == 1) {
            it += run_graphed(g, 1, iters, omega);
            if (it >= iters)
                break;
        }
        for (int nest = 0; nest < nests; ++nest) {
            check_deadline(g);
            const bool gpu = ((g->mask >> nest) & 1u) != 0;
            if (gpu)
                grid_ensure_device(g);
            xs.clear();
            const Validity before = g->valid;
            plan_before(it, nest, gpu, g->mode, g->valid, xs);
            if (gpu && g->level[nest] != OFL_LEVEL_K) {
                // The planner's whole-array decisions stand; hoisted ones run
                // here, outside the regions, per-iteration ones region by region.
                const bool per_iter = g->mode == OFL_XFER_PER_ITER;
                ins.clear();
                if (per_iter)
                    for (const Xfer &x : xs)
                        ins.push_back(x.array);
                else
                    grid_exec(g, xs);
                xs.clear();
                plan_after(it, nest, gpu, g->mode, g->valid, xs);
                int out = -1;
                for (const Xfer &x : xs)
                    out = x.array;  // per-iteration: the nest's written array, copied out by region
                if (!per_iter)
                    out = -1;
                gpu_nest_regions(g, nest, omega, per_iter, ins, out);
                // Per iteration, the regions moved only the rows they read (a
                // residual or copy-back region skips the boundary layer), so an
                // array that was not on the device before holds just those rows
                // there: the device copy is not whole and must not count as
                // valid. The host copy is whole (the rows came from it, and
                // written rows went back), so a later whole-array use re-sends it.
                if (per_iter)
                    for (int a : ins)
                        if (!before.dev[a])
                            g->valid.dev[a] = 0;
                continue;
            }
            grid_exec(g, xs);
            if (gpu)
                gpu_nest(g, nest, omega, fold && nest != kS);
            else
                cpu_nest(g, nest, omega);
            xs.clear();
            plan_after(it, nest, gpu, g->mode, g->valid, xs);
            grid_exec(g, xs);
            if (gpu && nest == kR && g->mode == OFL_XFER_PER_ITER) {
                // per-iteration placement: the residual scalar comes back every time
                hip_check(hipMemcpyAsync(&g->gosa_host, g->view.gosa, sizeof(double), hipMemcpyDeviceToHost,
                                         g->stream),
                          "hipMemcpyAsync(gosa)");
                g->gosa_on_dev = false;
            }
        }
    }
}

double grid_fetch_gosa(ofl_grid *g) {
    if (g->gosa_on_dev) {
        hip_check(hipMemcpyAsync(&g->gosa_host, g->view.gosa, sizeof(double), hipMemcpyDeviceToHost, g->stream),
                  "hipMemcpyAsync(gosa)");
        g->gosa_on_dev = false;
        g->pending = true;
    }
    grid_sync(g);
    return g->gosa_host;
}

namespace {

void encode_bf16(ofl_grid *g) {
    for (int a = 0; a < kNCoef; ++a) {
        const float *x = g->coef[a];
        const size_t n = g->n;
        float lo = std::numeric_limits<float>::infinity();
        float hi = -lo;
        bool exact = true;
        for (size_t t = 0; t < n; ++t) {
            const float v = x[t];
            lo = std::min(lo, v);
            hi = std::max(hi, v);
            uint32_t u;
            std::memcpy(&u, &v, sizeof u);
            if ((u & 0xffffu) != 0)
                exact = false;
        }
        float b = 0.f;
        if (g->fmt == OFL_COEF_BF16_OFFSET && !exact)
            b = static_cast<float>(0.5 * (static_cast<double>(lo) + static_cast<double>(hi)));
        g->bias[a] = b;
        g->enc[a].resize(n);
        cpu_encode_bf16(x, n, b, g->enc[a].data());
    }
}

}  // namespace

// p and wrk2 exchange device buffers: the copy-back of a fused iteration.
void grid_swap_p_wrk2(ofl_grid *g) {
    std::swap(g->lay.off[OFL_ARR_P], g->lay.off[OFL_ARR_WRK2]);
    std::swap(g->view.p, g->view.wrk2);
    g->swap_epoch += 1;
}

// Give the device wrk2 p's boundary (both buffers then share it), once per upload of p.
void grid_sync_wrk2_boundary(ofl_grid *g) {
    if (g->wrk2_boundary_ok)
        return;
    launch_copy(grid_array_ptr(g, OFL_ARR_WRK2), grid_array_ptr(g, OFL_ARR_P), g->lay.elems * sizeof(float), g->stream);
    g->wrk2_boundary_ok = true;
    g->pending = true;
}

void grid_sync(ofl_grid *g) {
    if (!g->dev_ready)
        return;
    hip_check(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    harvest_events(g);
    g->pending = false;
}

void grid_exec(ofl_grid *g, const std::vector<Xfer> &xs) {
    for (const Xfer &x : xs) {
        TraceRange range(kXferRange[x.dir != 0 ? 1 : 0][x.array]);
        grid_ensure_device(g);
        const size_t eb = array_elem_bytes(g, x.array);
        const size_t bytes = g->n * eb;
        void *staging = g->block + g->lay.staging_off;
        void *arr = grid_array_ptr(g, x.array);
        if (x.dir == 0) {
            hip_check(hipMemcpyAsync(staging, host_src(g, x.array), bytes, hipMemcpyHostToDevice, g->stream),
                      "hipMemcpyAsync(host->device)");
            const bool coef = x.array < kNCoef;
            launch_pack(staging, arr, g->I, g->J, g->K, coef ? g->lay.crow : g->I,
                        coef ? g->lay.cpitch : g->lay.pitch,
                        static_cast<long long>(coef ? g->lay.cplane : g->lay.plane), static_cast<int>(eb), g->stream);
            if (x.array == OFL_ARR_P || x.array == OFL_ARR_WRK2)
                g->wrk2_boundary_ok = false;
            g->stats.h2d_count += 1;
            g->stats.h2d_bytes += bytes;
        } else {
            void *dst = x.array == OFL_ARR_P ? static_cast<void *>(g->p) : static_cast<void *>(g->wrk2);
            launch_unpack(arr, staging, g->I, g->J, g->K, g->lay.pitch, static_cast<long long>(g->lay.plane),
                          static_cast<int>(eb), g->stream);
            hip_check(hipMemcpyAsync(dst, staging, bytes, hipMemcpyDeviceToHost, g->stream),
                      "hipMemcpyAsync(device->host)");
            g->stats.d2h_count += 1;
            g->stats.d2h_bytes += bytes;
        }
        g->pending = true;
    }
}

namespace {

// The program's loop statements in order: the iteration loop, then k, j, i of S, R, C.
void loop_table(const ofl_grid *g, ofl_loop_info *out) {
    out[0] = {-1, -1, 0, 0};  // trip n reads the p that trip n-1 wrote: no region can open here
    const int extent[3] = {g->K - 2, g->J - 2, g->I - 2};
    for (int n = 0; n < 3; ++n)
        for (int l = 0; l < 3; ++l)
            out[1 + 3 * n + l] = {n, l, extent[l], 1};
}

void check_regions(unsigned mask, const int *level, int xfer_mode) {
    if (mask > OFL_MASK_ALL_GPU)
        fail(OFL_EINVAL, "mask has bits above bit 2");
    if (xfer_mode != OFL_XFER_PER_ITER && xfer_mode != OFL_XFER_HOISTED)
        fail(OFL_EINVAL, "unknown xfer_mode");
    for (int n = 0; n < 3; ++n)
        if (level[n] < OFL_LEVEL_K || level[n] > OFL_LEVEL_I)
            fail(OFL_EINVAL, "unknown region level");
}

}  // namespace

// Loop gene -> regions: the gene's bits follow the loops that pass the screen,
// in program order; a nest's region opens at its outermost offloaded loop.
int loop_gene_bits(const ofl_grid *g) {
    ofl_loop_info t[OFL_NLOOPS];
    loop_table(g, t);
    int bits = 0;
    for (const ofl_loop_info &x : t)
        bits += x.parallel;
    return bits;
}

void decode_loop_gene(const ofl_grid *g, uint32_t gene, unsigned *mask, int level[3]) {
    ofl_loop_info t[OFL_NLOOPS];
    loop_table(g, t);
    *mask = 0;
    for (int n = 0; n < 3; ++n)
        level[n] = OFL_LEVEL_K;
    int b = 0;
    bool opened[3] = {false, false, false};
    for (const ofl_loop_info &x : t) {
        if (!x.parallel)
            continue;
        const bool on = ((gene >> b) & 1u) != 0;
        b += 1;
        if (on && !opened[x.nest]) {
            opened[x.nest] = true;
            *mask |= 1u << x.nest;
            level[x.nest] = x.level;
        }
    }
}

}  // namespace ofl

using namespace ofl;

extern "C" {

const char *ofl_last_error(void) { return t_last_error.c_str(); }

const char *ofl_version(void) { return "ofl 0.1.0 (gfx950)"; }

int ofl_grid_device_bytes(int I, int J, int K, int coef_format, int row_align, size_t *bytes) {
    return guarded(nullptr, [&] {
        if (!bytes)
            fail(OFL_EINVAL, "bytes is NULL");
        if (I < 3 || J < 3 || K < 3)
            fail(OFL_EINVAL, "every grid dimension must be >= 3");
        if (coef_format < OFL_COEF_F32 || coef_format > OFL_COEF_BF16_OFFSET)
            fail(OFL_EINVAL, "unknown coef_format");
        if (!row_align_valid(row_align))
            fail(OFL_EINVAL, "row_align must be 0, 4, 8, 16 or 32");
        *bytes = make_layout(I, J, K, coef_format, row_align).total;
    });
}

int ofl_grid_create(const ofl_grid_desc *d, ofl_grid **out) {
    return guarded(nullptr, [&] {
        if (!d || !out)
            fail(OFL_EINVAL, "desc and out must not be NULL");
        if (d->I < 3 || d->J < 3 || d->K < 3)
            fail(OFL_EINVAL, "every grid dimension must be >= 3");
        const long long n = static_cast<long long>(d->I) * d->J * d->K;
        if (n > (1LL << 36) || static_cast<long long>(round_up(d->I, kPitchAlign)) * d->J * d->K > (1LL << 40))
            fail(OFL_EINVAL, "grid too large");
        if (static_cast<long long>(d->J) * d->K > 0x7fffffffLL / 4)
            fail(OFL_EINVAL, "grid has too many rows");
        if (d->coef_format < OFL_COEF_F32 || d->coef_format > OFL_COEF_BF16_OFFSET)
            fail(OFL_EINVAL, "unknown coef_format");
        if (d->sum_mode != OFL_SUM_F64 && d->sum_mode != OFL_SUM_KAHAN_F32)
            fail(OFL_EINVAL, "unknown sum_mode");
        if (!d->p || !d->wrk2)
            fail(OFL_EINVAL, "p and wrk2 must not be NULL");
        for (int a = 0; a < kNCoef; ++a)
            if (!d->coef[a])
                fail(OFL_EINVAL, "every coefficient array must be given");
        if (!row_align_valid(d->row_align))
            fail(OFL_EINVAL, "row_align must be 0, 4, 8, 16 or 32");
        if (d->dev_arena && (reinterpret_cast<uintptr_t>(d->dev_arena) % 256) != 0)
            fail(OFL_EINVAL, "dev_arena must be 256-byte aligned");
        std::unique_ptr<ofl_grid> g(new ofl_grid);
        g->I = d->I;
        g->J = d->J;
        g->K = d->K;
        g->n = static_cast<size_t>(n);
        g->fmt = d->coef_format;
        g->sum_mode = d->sum_mode;
        g->p = d->p;
        g->wrk2 = d->wrk2;
        for (int a = 0; a < kNCoef; ++a)
            g->coef[a] = d->coef[a];
        g->user_stream = d->stream;
        g->arena = d->dev_arena;
        g->arena_bytes = d->dev_arena_bytes;
        g->want_device = d->device;
        g->row_align = d->row_align;
        g->tile = default_tile(d->I, d->coef_format, 0);
        if (g->fmt != OFL_COEF_F32)
            encode_bf16(g.get());
        *out = g.release();
    });
}

void ofl_grid_destroy(ofl_grid *g) {
    if (!g)
        return;
    if (g->dev_ready) {
        (void)hipSetDevice(g->device);
        (void)hipStreamSynchronize(g->stream);
        for (hipEvent_t e : g->ev)
            (void)hipEventDestroy(e);
        if (g->fused_parts)
            (void)hipFree(g->fused_parts);
        if (g->region_sums)
            (void)hipFree(g->region_sums);
        grid_drop_graphs(g);
        if (g->own_block)
            (void)hipFree(g->block);
        if (g->own_stream)
            (void)hipStreamDestroy(g->stream);
    }
    delete g;
}

int ofl_set_offload_mask(ofl_grid *g, unsigned mask, int xfer_mode) {
    return grid_call(g, [&] {
        if (mask > OFL_MASK_ALL_GPU)
            fail(OFL_EINVAL, "mask has bits above bit 2");
        if (xfer_mode != OFL_XFER_PER_ITER && xfer_mode != OFL_XFER_HOISTED)
            fail(OFL_EINVAL, "unknown xfer_mode");
        g->mask = mask;
        g->mode = xfer_mode;
        for (int n = 0; n < 3; ++n)
            g->level[n] = OFL_LEVEL_K;
    });
}

int ofl_loop_table(const ofl_grid *g, ofl_loop_info out[OFL_NLOOPS]) {
    return guarded(nullptr, [&] {
        if (!g || !out)
            fail(OFL_EINVAL, "NULL argument");
        loop_table(g, out);
    });
}

int ofl_set_loop_gene(ofl_grid *g, uint32_t gene, int xfer_mode) {
    return grid_call(g, [&] {
        const int bits = loop_gene_bits(g);
        if (bits < 32 && (gene >> bits) != 0)
            fail(OFL_EINVAL, "gene has bits beyond the loops that pass the screen");
        unsigned mask = 0;
        int level[3];
        decode_loop_gene(g, gene, &mask, level);
        check_regions(mask, level, xfer_mode);
        g->mask = mask;
        g->mode = xfer_mode;
        for (int n = 0; n < 3; ++n)
            g->level[n] = level[n];
    });
}

int ofl_set_regions(ofl_grid *g, unsigned mask, const int level[3], int xfer_mode) {
    return grid_call(g, [&] {
        if (!level)
            fail(OFL_EINVAL, "NULL level");
        check_regions(mask, level, xfer_mode);
        g->mask = mask;
        g->mode = xfer_mode;
        for (int n = 0; n < 3; ++n)
            g->level[n] = level[n];
    });
}

int ofl_get_regions(const ofl_grid *g, unsigned *mask, int level[3], int *xfer_mode) {
    return guarded(nullptr, [&] {
        if (!g || !mask || !level || !xfer_mode)
            fail(OFL_EINVAL, "NULL argument");
        *mask = g->mask;
        *xfer_mode = g->mode;
        for (int n = 0; n < 3; ++n)
            level[n] = g->level[n];
    });
}

int ofl_jacobi_run(ofl_grid *g, int iters, float omega, double *gosa_out) {
    return grid_call(g, [&] {
        if (iters < 0)
            fail(OFL_EINVAL, "iters must be >= 0");
        if (!std::isfinite(omega) || omega == 0.f)
            fail(OFL_EINVAL, "omega must be finite and non-zero");
        if (g->batch_refs > 0 && g->mask != OFL_MASK_ALL_GPU)
            fail(OFL_ESTATE, "a grid inside a batch runs with every nest on the GPU");
        if (iters == 0) {
            if (gosa_out)
                *gosa_out = std::numeric_limits<double>::quiet_NaN();
            return;
        }
        grid_run_loop(g, iters, omega, 3);
        if (!g->in_region) {
            std::vector<Xfer> xs;
            plan_sync_host(iters, g->valid, xs);
            grid_exec(g, xs);
        }
        const double gosa = grid_fetch_gosa(g);
        if (gosa_out)
            *gosa_out = gosa;
    });
}

int ofl_jacobi_run_static(ofl_grid *g, int iters, float omega, double *gosa_out) {
    return grid_call(g, [&] {
        if (iters < 0)
            fail(OFL_EINVAL, "iters must be >= 0");
        if (!std::isfinite(omega) || omega == 0.f)
            fail(OFL_EINVAL, "omega must be finite and non-zero");
        if (!g->dev_ready || !g->in_region)
            fail(OFL_ESTATE, "ofl_jacobi_run_static needs the grid resident: open a data region (ofl_data_enter) first");
        if (g->mask != OFL_MASK_ALL_GPU || g->mode != OFL_XFER_HOISTED || !grid_whole_nests(g))
            fail(OFL_ENOTSUP, "ofl_jacobi_run_static runs gene 111 with hoisted transfers and whole nests only");
        if (g->batch_refs > 0)
            fail(OFL_ESTATE, "the grid belongs to a batch");
        if ((g->fusion & OFL_FUSE_RESIDUAL) == 0)
            fail(OFL_ENOTSUP, "ofl_jacobi_run_static runs the fused residual: set OFL_FUSE_RESIDUAL (ofl_set_fusion)");
        if (g->profiling)
            fail(OFL_ENOTSUP, "profiling creates HIP events; switch it off for ofl_jacobi_run_static");
        // two buffers of one partial per sweep wave
        const long long need = 2 * sweep_waves(g->I, g->J, g->K, g->tile);
        if (need > kStaticScratchParts)
            fail(OFL_EINVAL, "the grid's sweep needs " + std::to_string(need) +
                                 " residual partials, more than the static scratch holds (" +
                                 std::to_string(kStaticScratchParts) + "); use a tile with longer k-chunks, or ofl_jacobi_run");
        if (iters == 0) {
            if (gosa_out)
                *gosa_out = std::numeric_limits<double>::quiet_NaN();
            return;
        }
        grid_ensure_device(g);  // device state exists: selects the grid's device only
        run_fused(g, iters, omega, static_scratch(g->device));
        const double gosa = grid_fetch_gosa(g);
        if (gosa_out)
            *gosa_out = gosa;
    });
}

int ofl_residual(ofl_grid *g, double *gosa_out) {
    return grid_call(g, [&] {
        if (!gosa_out)
            fail(OFL_EINVAL, "gosa_out must not be NULL");
        grid_run_loop(g, 1, 1.0f, 2);
        *gosa_out = grid_fetch_gosa(g);
    });
}

int ofl_data_enter(ofl_grid *g) {
    return grid_call(g, [&] {
        if (g->in_region)
            fail(OFL_ESTATE, "data region already open");
        if (g->mask != 0) {
            grid_ensure_device(g);
            std::vector<Xfer> xs;
            plan_enter(g->mask, g->valid, xs);
            grid_exec(g, xs);
            grid_sync(g);
        }
        g->in_region = true;
    });
}

int ofl_update_host(ofl_grid *g) {
    return grid_call(g, [&] {
        std::vector<Xfer> xs;
        plan_sync_host(-1, g->valid, xs);
        grid_exec(g, xs);
        grid_sync(g);
    });
}

int ofl_data_exit(ofl_grid *g) {
    return grid_call(g, [&] {
        if (!g->in_region)
            fail(OFL_ESTATE, "no data region is open");
        std::vector<Xfer> xs;
        plan_sync_host(-1, g->valid, xs);
        grid_exec(g, xs);
        grid_sync(g);
        g->in_region = false;
    });
}

int ofl_grid_coef_bias(const ofl_grid *g, float bias[12]) {
    return guarded(nullptr, [&] {
        if (!g || !bias)
            fail(OFL_EINVAL, "NULL argument");
        for (int a = 0; a < kNCoef; ++a)
            bias[a] = g->bias[a];
    });
}

int ofl_set_fusion(ofl_grid *g, unsigned flags) {
    return grid_call(g, [&] {
        if (flags & ~static_cast<unsigned>(OFL_FUSE_RESIDUAL | OFL_FUSE_COPYBACK_SWAP))
            fail(OFL_EINVAL, "unknown fusion bits");
        if (flags != 0 && g->batch_refs > 0)
            fail(OFL_ESTATE, "a grid inside a batch cannot swap its buffers; destroy the batch first");
        if ((flags & OFL_FUSE_RESIDUAL) && g->sum_mode != OFL_SUM_F64)
            fail(OFL_ENOTSUP, "the fused residual sums in FP64 only; this grid asks for compensated FP32");
        g->fusion = flags;
        if (!g->tile_chosen)
            g->tile = default_tile(g->I, g->fmt, flags);
    });
}

int ofl_set_tile(ofl_grid *g, const ofl_tile *tile) {
    return grid_call(g, [&] {
        std::string why;
        if (!tile)
            fail(OFL_EINVAL, "tile is NULL");
        if (!tile_valid(*tile, &why))
            fail(OFL_EINVAL, why);
        if (tile->vec == 8 && make_layout(g->I, g->J, g->K, g->fmt, g->row_align).pitch % 8 != 0)
            fail(OFL_EINVAL, "tile.vec 8 needs a row pitch that is a multiple of 8 elements (row_align 0, 8, 16 or 32)");
        g->tile = to_cfg(*tile);
        g->tile_chosen = true;
    });
}

int ofl_get_tile(const ofl_grid *g, ofl_tile *tile) {
    return guarded(nullptr, [&] {
        if (!g || !tile)
            fail(OFL_EINVAL, "NULL argument");
        *tile = to_tile(g->tile);
    });
}

int ofl_set_profiling(ofl_grid *g, int on) {
    return grid_call(g, [&] {
        if (g->dev_ready)
            grid_sync(g);
        g->profiling = on != 0;
    });
}

int ofl_set_profiled_nests(ofl_grid *g, unsigned nests) {
    return grid_call(g, [&] {
        if (nests > OFL_MASK_ALL_GPU)
            fail(OFL_EINVAL, "nests has bits above bit 2");
        if (g->dev_ready)
            grid_sync(g);
        g->prof_nests = nests;
    });
}

int ofl_get_stats(const ofl_grid *g, ofl_stats *out) {
    return guarded(nullptr, [&] {
        if (!g || !out)
            fail(OFL_EINVAL, "NULL argument");
        *out = g->stats;
    });
}

int ofl_reset_stats(ofl_grid *g) {
    return grid_call(g, [&] {
        if (g->dev_ready)
            grid_sync(g);
        g->stats = ofl_stats{};
    });
}

int ofl_plan(unsigned mask, int xfer_mode, int iters, int sync_host_at_end, uint8_t host_valid[14],
             uint8_t dev_valid[14], ofl_xfer *out, int cap, int *count) {
    const Program &prog = jacobi_program();
    ofl_nest_vars nv[3];
    for (int n = 0; n < 3; ++n)
        nv[n] = {prog.nests[n].reads, prog.nests[n].writes, prog.nests[n].partial};
    return ofl_plan_nests(nv, prog.nnests, prog.narrays, prog.live_after, mask, xfer_mode, iters, sync_host_at_end,
                          host_valid, dev_valid, out, cap, count);
}

int ofl_plan_nests(const ofl_nest_vars *nests, int nnests, int narrays, uint32_t live_after, unsigned mask,
                   int xfer_mode, int iters, int sync_host_at_end, uint8_t *host_valid, uint8_t *dev_valid,
                   ofl_xfer *out, int cap, int *count) {
    return guarded(nullptr, [&] {
        if (!nests || nnests < 1 || nnests > kMaxNests || narrays < 1 || narrays > kMaxArrays)
            fail(OFL_EINVAL, "nests must hold 1..8 entries over 1..32 arrays");
        const uint32_t all = narrays == 32 ? 0xffffffffu : ((1u << narrays) - 1u);
        Program prog{};
        prog.nnests = nnests;
        prog.narrays = narrays;
        prog.live_after = live_after;
        for (int n = 0; n < nnests; ++n) {
            const ofl_nest_vars &x = nests[n];
            if (((x.reads | x.writes | x.partial) & ~all) != 0)
                fail(OFL_EINVAL, "a nest names an array beyond narrays");
            if ((x.partial & ~x.writes) != 0)
                fail(OFL_EINVAL, "a partial write must also be a write");
            prog.nests[n] = {x.reads, x.writes, x.partial};
        }
        if ((live_after & ~all) != 0)
            fail(OFL_EINVAL, "live_after names an array beyond narrays");
        if ((mask >> nnests) != 0)
            fail(OFL_EINVAL, "mask has bits beyond the nests");
        if (xfer_mode != OFL_XFER_PER_ITER && xfer_mode != OFL_XFER_HOISTED)
            fail(OFL_EINVAL, "unknown xfer_mode");
        if (iters < 0 || !host_valid || !dev_valid || !count || cap < 0 || (cap > 0 && !out))
            fail(OFL_EINVAL, "bad iters, state or output arguments");
        Validity v = fresh_validity();
        for (int a = 0; a < narrays; ++a) {
            v.host[a] = host_valid[a] ? 1 : 0;
            v.dev[a] = dev_valid[a] ? 1 : 0;
            if (!v.host[a] && !v.dev[a])
                fail(OFL_EINVAL, "an array is valid on neither side");
        }
        std::vector<Xfer> xs;
        for (int it = 0; it < iters; ++it)
            for (int nest = 0; nest < nnests; ++nest) {
                const bool gpu = ((mask >> nest) & 1u) != 0;
                plan_before(prog, it, nest, gpu, xfer_mode, v, xs);
                plan_after(prog, it, nest, gpu, xfer_mode, v, xs);
            }
        if (sync_host_at_end && iters > 0)
            plan_sync_host(prog, iters, v, xs);
        *count = static_cast<int>(xs.size());
        for (int a = 0; a < narrays; ++a) {
            host_valid[a] = v.host[a];
            dev_valid[a] = v.dev[a];
        }
        const int m = std::min(cap, static_cast<int>(xs.size()));
        for (int t = 0; t < m; ++t)
            out[t] = ofl_xfer{xs[t].iter, xs[t].nest, xs[t].when, xs[t].array, xs[t].dir};
        if (static_cast<int>(xs.size()) > cap)
            fail(OFL_ENOMEM, "out has fewer entries than the plan");
    });
}

int ofl_program_vars(ofl_nest_vars out[3], uint32_t *live_after) {
    return guarded(nullptr, [&] {
        if (!out || !live_after)
            fail(OFL_EINVAL, "NULL argument");
        const Program &prog = jacobi_program();
        for (int n = 0; n < 3; ++n)
            out[n] = {prog.nests[n].reads, prog.nests[n].writes, prog.nests[n].partial};
        *live_after = prog.live_after;
    });
}

int ofl_device_copy(void *dst, const void *src, size_t bytes, void *stream) {
    return guarded(nullptr, [&] {
        if (!dst || !src)
            fail(OFL_EINVAL, "NULL pointer");
        if (bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0 ||
            reinterpret_cast<uintptr_t>(src) % 16 != 0)
            fail(OFL_EINVAL, "bytes and both pointers must be multiples of 16");
        launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream));
    });
}

int ofl_device_stream(const float *const *src32, int n32, const uint16_t *const *src16, int n16, float *dst,
                      size_t n, void *stream) {
    return guarded(nullptr, [&] {
        if (!dst || (n32 > 0 && !src32) || (n16 > 0 && !src16))
            fail(OFL_EINVAL, "NULL pointer");
        if (!((n32 == 13 && n16 == 0) || (n32 == 1 && n16 == 12)))
            fail(OFL_ENOTSUP, "stream patterns: 13 FP32 sources, or 1 FP32 and 12 bfloat16 sources");
        if (n % 4 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
            fail(OFL_EINVAL, "n must be a multiple of 4 and dst 16-byte aligned");
        for (int t = 0; t < n32; ++t)
            if (!src32[t] || reinterpret_cast<uintptr_t>(src32[t]) % 16 != 0)
                fail(OFL_EINVAL, "every FP32 source must be given and 16-byte aligned");
        for (int t = 0; t < n16; ++t)
            if (!src16[t] || reinterpret_cast<uintptr_t>(src16[t]) % 8 != 0)
                fail(OFL_EINVAL, "every bfloat16 source must be given and 8-byte aligned");
        launch_stream(src32, n32, src16, n16, dst, n, static_cast<hipStream_t>(stream));
    });
}

}  // extern "C"
