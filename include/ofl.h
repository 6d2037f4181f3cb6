/*
 * ofl.h -- C ABI of the offloaded Jacobi loop-nest library for MI355X (gfx950).
 *
 * The paper's loop-offload method (Sec. 3.2.1, Sec. 4.2.2) takes a CPU
 * program, gives every parallelisable loop nest one gene bit (1 = run it on
 * the GPU, 0 = leave it on the CPU), moves variables between host and device
 * only where a nest on one side reads what the other side wrote, and places
 * those transfers at the outermost loop level that allows it instead of inside
 * the inner loops. The program offloaded here is a 3D variable-coefficient
 * 19-point Jacobi relaxation with three loop nests per iteration:
 *
 *   S  sweep      wrk2 = p + omega*ss on the interior, where
 *                 ss = (a3*s0 - p)*bnd and s0 is the 19-point sum
 *                   a0 p(i+1) + a1 p(j+1) + a2 p(k+1) + c0 p(i-1) + c1 p(j-1) + c2 p(k-1)
 *                 + b0 [p(i+1,j+1) - p(i+1,j-1) - p(i-1,j+1) + p(i-1,j-1)]
 *                 + b1 [p(j+1,k+1) - p(j-1,k+1) - p(j+1,k-1) + p(j-1,k-1)]
 *                 + b2 [p(i+1,k+1) - p(i-1,k+1) - p(i+1,k-1) + p(i-1,k-1)] + wrk1
 *                 (every coefficient at the centre point, p the old iterate)
 *   R  residual   gosa = sum over the interior of ((wrk2 - p)/omega)^2
 *   C  copy-back  p = wrk2 on the interior
 *
 * The interior is {1..I-2} x {1..J-2} x {1..K-2}; the outer one-cell layer of
 * p is a fixed (Dirichlet) boundary.
 *
 * Host array layout: I*J*K floats, linear index i + I*(j + J*k) (i fastest).
 * Coefficient order everywhere: a0 a1 a2 a3 b0 b1 b2 c0 c1 c2 bnd wrk1.
 *
 * Errors: every call returns an OFL_* status. On failure the outputs are left
 * untouched and ofl_last_error() (per thread) describes the cause. A failing
 * HIP call makes the handle unusable (OFL_EDEVICE is sticky): after it only
 * the destroy call is valid. No C++ exception crosses this interface.
 * Threads: one handle must not be used by two threads at once; separate
 * handles may run concurrently.
 */
#ifndef OFL_H
#define OFL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define OFL_OK 0
#define OFL_EINVAL (-1)  /* bad argument */
#define OFL_ENOMEM (-2)  /* host or device memory exhausted, arena too small */
#define OFL_EDEVICE (-3) /* a HIP call failed or no GPU is present (sticky) */
#define OFL_ESTATE (-4)  /* call not valid in the handle's current state */
#define OFL_ENOTSUP (-5) /* combination not supported */

/* ---- offload gene: one bit per loop nest, 1 = GPU, 0 = CPU (Sec. 3.2.1) --- */
#define OFL_NEST_SWEEP 1u
#define OFL_NEST_RESIDUAL 2u
#define OFL_NEST_COPYBACK 4u
#define OFL_MASK_ALL_CPU 0u
#define OFL_MASK_ALL_GPU 7u

/* ---- transfer placement (Sec. 3.2.1, Sec. 4.2.2) ------------------------ */
/* PER_ITER: every GPU nest copies in all it reads and copies out all it
 * writes, each time it runs (transfers inside the loop).
 * HOISTED: an array moves only when the side that needs it does not hold a
 * valid copy, so read-only arrays move once and nothing moves per iteration
 * when every nest is on the GPU (transfers at the outermost level). */
#define OFL_XFER_PER_ITER 0
#define OFL_XFER_HOISTED 1

/* ---- device storage of the twelve read-only arrays ---------------------- */
#define OFL_COEF_F32 0          /* FP32 as given */
#define OFL_COEF_BF16 1         /* bfloat16, round to nearest even */
#define OFL_COEF_BF16_OFFSET 2  /* per-array FP32 bias + bfloat16 of (x - bias) */

/* ---- residual accumulation ---------------------------------------------- */
#define OFL_SUM_F64 0       /* squares summed in FP64 */
#define OFL_SUM_KAHAN_F32 1 /* per-thread compensated (Neumaier) FP32, FP64 across threads */

/* ---- array ids (transfer plans and statistics) -------------------------- */
enum {
    OFL_ARR_A0 = 0, OFL_ARR_A1, OFL_ARR_A2, OFL_ARR_A3,
    OFL_ARR_B0, OFL_ARR_B1, OFL_ARR_B2,
    OFL_ARR_C0, OFL_ARR_C1, OFL_ARR_C2,
    OFL_ARR_BND, OFL_ARR_WRK1,
    OFL_ARR_P = 12, OFL_ARR_WRK2 = 13,
    OFL_NARRAYS = 14
};

/* ---- grid description ---------------------------------------------------- */
typedef struct ofl_grid ofl_grid;

typedef struct ofl_grid_desc {
    int I, J, K;            /* points per axis, each >= 3; I fastest in memory */
    int coef_format;        /* OFL_COEF_* */
    int sum_mode;           /* OFL_SUM_* */
    float *p;               /* host, I*J*K: initial iterate in, result out */
    float *wrk2;            /* host, I*J*K: scratch; contents unspecified after a run */
    const float *coef[12];  /* host, I*J*K each, read-only; order a0..a3 b0..b2 c0..c2 bnd wrk1 */
    void *stream;           /* hipStream_t to launch on, borrowed; NULL: the library makes one */
    void *dev_arena;        /* optional caller-owned device memory (e.g. from PyTorch), 256-byte
                               aligned, at least ofl_grid_device_bytes(I, J, K, coef_format,
                               row_align) bytes; NULL: hipMalloc */
    size_t dev_arena_bytes; /* size of dev_arena */
    int device;             /* HIP device ordinal; -1: the device current at creation */
    int row_align;          /* elements every device row is padded to: 0 for a 128-byte line (32 FP32 or
                               64 bfloat16 elements), else 4, 8, 16 or 32. Short rows waste less memory
                               with a small alignment, and a batch runs such grids in packed rows
                               (ofl_batch_create). Results do not depend on it. */
} ofl_grid_desc;

/* Device bytes a grid of this shape, format and row alignment (as in
 * desc.row_align: 0, 4, 8, 16 or 32) needs: the size a dev_arena must have.
 * A compact row alignment can need more than the default one, because it also
 * pads every plane to 64 elements. Returns OFL_EINVAL for a dimension below 3,
 * an unknown format or row alignment, or a NULL bytes. */
int ofl_grid_device_bytes(int I, int J, int K, int coef_format, int row_align, size_t *bytes);

/* Create a grid handle over the caller's host arrays (the CPU program's
 * variables, Sec. 4.2.2). The host arrays are borrowed and must outlive the
 * handle; they are read at creation (bfloat16 formats encode the twelve
 * read-only arrays into library-owned host copies here) and whenever the
 * transfer plan moves them. Device memory is taken only when a GPU nest first
 * needs it, so an all-CPU mask runs without a GPU. The initial mask is
 * OFL_MASK_ALL_GPU with hoisted transfers. EINVAL on a NULL pointer, a
 * dimension below 3 or an unknown format/sum mode; ENOMEM when host memory
 * runs out. */
int ofl_grid_create(const ofl_grid_desc *desc, ofl_grid **out);

/* Release the handle, its device buffers (unless they live in the caller's
 * arena) and its stream (unless borrowed). NULL is ignored. */
void ofl_grid_destroy(ofl_grid *g);

/* Choose the device of each loop nest: bit0 sweep, bit1 residual, bit2
 * copy-back, bit = 1 -> GPU (the gene of Sec. 3.2.1 / Sec. 4.2.2), and the
 * transfer placement (OFL_XFER_*). Takes effect at the next run; data already
 * on either side stays valid. EINVAL for bits above 2 or an unknown mode. */
int ofl_set_offload_mask(ofl_grid *g, unsigned mask, int xfer_mode);

/* ---- one gene bit per loop statement (Sec. 4.2.2) -------------------------
 * The offloaded program's loop statements, outermost first: the iteration loop,
 * then the k, j and i loops of each nest (S, R, C). Offloading a loop starts a
 * GPU region there; every loop inside the region is parallel in the kernel,
 * and the loops outside it stay on the host, which then launches one region
 * per trip. So a GPU nest's region opens at one of three levels:
 *   OFL_LEVEL_K  the whole nest is one launch (what ofl_set_offload_mask sets);
 *   OFL_LEVEL_J  the host loops over k, one launch per interior plane;
 *   OFL_LEVEL_I  the host loops over k and j, one launch per interior row.
 * Results do not depend on the level (p is bitwise identical; gosa is summed
 * per region, then over regions in order, both in FP64). Transfers: hoisted,
 * they stay outside the iteration loop as for whole-nest regions; per
 * iteration, every region copies in the rows it reads (for S, p's rows j-1..j+1
 * of planes k-1..k+1) and copies out the rows it writes, and each residual
 * region's FP64 sum comes back to the host, which adds them. The fused paths
 * (ofl_set_fusion) apply only when every GPU region is a whole nest; a batch
 * always runs whole nests. */
enum { OFL_LEVEL_K = 0, OFL_LEVEL_J = 1, OFL_LEVEL_I = 2 };
#define OFL_NLOOPS 10

typedef struct ofl_loop_info {
    int nest;      /* -1 for the iteration loop, else 0 S, 1 R, 2 C */
    int level;     /* -1 for the iteration loop, else OFL_LEVEL_* */
    int extent;    /* trip count on this grid (the iteration loop: 0, set by each run) */
    int parallel;  /* 1 if a GPU region can open at this loop (the screen of Sec. 4.2.2):
                      0 for the iteration loop, whose trips read what the previous one wrote */
} ofl_loop_info;

/* The loop statements of the program on this grid, OFL_NLOOPS entries in
 * program order: index 0 the iteration loop, 1 + 3*nest + level the others.
 * EINVAL on NULL. */
int ofl_loop_table(const ofl_grid *g, ofl_loop_info out[OFL_NLOOPS]);

/* Apply a loop gene: bit b belongs to the b-th loop of ofl_loop_table that
 * passes the screen, in table order (9 bits here: S k,j,i, R k,j,i, C k,j,i).
 * A nest runs on the GPU if one of its bits is 1, its region opening at the
 * outermost such loop; bits inside an offloaded loop change nothing (they were
 * parallel already). EINVAL for bits beyond the gene length or an unknown
 * placement. */
int ofl_set_loop_gene(ofl_grid *g, uint32_t gene, int xfer_mode);

/* Set the regions directly: mask as in ofl_set_offload_mask, level[n] the
 * level of nest n's region (ignored for CPU nests); and read them back.
 * EINVAL for an unknown mask bit, level or placement. */
int ofl_set_regions(ofl_grid *g, unsigned mask, const int level[3], int xfer_mode);
int ofl_get_regions(const ofl_grid *g, unsigned *mask, int level[3], int *xfer_mode);

/* Run iters x (S, R, C), each nest on the device its gene bit names, with the
 * transfers the planner derives (Sec. 4.2.2: a CPU-written variable that the
 * GPU reads moves host->device; a GPU-written variable the CPU references
 * moves device->host). On return the caller's p holds the new iterate, unless
 * a data region is open (ofl_data_enter), in which case p stays on the device
 * until ofl_update_host/ofl_data_exit. *gosa_out (nullable) receives R of the
 * last iteration, i.e. the residual of the iterate before the last update;
 * iters == 0 leaves p alone and gives NaN. EINVAL for iters < 0 or omega == 0
 * or non-finite; EDEVICE when a GPU nest is requested and no GPU is usable. */
int ofl_jacobi_run(ofl_grid *g, int iters, float omega, double *gosa_out);

/* ofl_jacobi_run for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): it
 * calls no hipMalloc, hipFree, event or graph creation. It runs the fused
 * iteration (see ofl_set_fusion) with the sweep's per-wave residual partials
 * (two buffers: even and odd iterations) in a library-owned device array of
 * 2^19 FP64 slots (4 MiB per device, held until the process ends) instead of a
 * buffer the library allocates; results
 * are bitwise those of ofl_jacobi_run on the same grid and tile. Preconditions,
 * each refused before any work: the grid is resident (ofl_data_enter done,
 * ESTATE otherwise), gene 111 with hoisted transfers and whole nests (ENOTSUP),
 * OFL_FUSE_RESIDUAL set (ENOTSUP), profiling off (ENOTSUP), not inside a batch
 * (ESTATE), and a sweep of at most 2^18 waves for the grid's tile (EINVAL: a
 * tile with longer k-chunks needs fewer). Every call on one
 * device shares that array, so calls that overlap in time on one device (two
 * host threads, or two streams) race and give wrong residuals; serialise them.
 * p and gosa are as for ofl_jacobi_run; a data region stays open. */
int ofl_jacobi_run_static(ofl_grid *g, int iters, float omega, double *gosa_out);

/* Residual of the current iterate without changing it: S with omega = 1 into
 * wrk2, then R; no copy-back. Uses the devices of the current mask. The paper
 * defines no such call: it is the offloaded program's own residual nest, run
 * once on the current iterate, for a caller that wants a convergence check
 * outside the iteration loop. */
int ofl_residual(ofl_grid *g, double *gosa_out);

/* Data region (the hoisting of Sec. 3.2.1 across calls, like an OpenACC data
 * region with "present" inside, Sec. 4.3.1): enter copies to the device every
 * array the current mask's GPU nests read and keeps the results of later runs
 * on the device; update_host brings the caller's p (and wrk2 if its last valid
 * copy is on the device) up to date without leaving; exit does the same and
 * closes the region. ESTATE when entering twice or exiting when not inside. */
int ofl_data_enter(ofl_grid *g);
int ofl_update_host(ofl_grid *g);
int ofl_data_exit(ofl_grid *g);

/* ---- fusion of adjacent GPU nests ---------------------------------------- */
/* Extends the hoisting idea of Sec. 3.2.1 from PCIe to HBM traffic: when every
 * nest runs on the GPU (gene 111) with hoisted transfers, the sweep can also
 * produce the residual (OFL_FUSE_RESIDUAL: the residual nest's own terms,
 * (wrk2 - p) in FP32 squared and summed in FP64, one partial per wave, then a
 * fixed-order sum; the sum of one iteration's partials runs in the first
 * work-group of the next iteration's sweep launch, the last iteration's after
 * the loop), and the copy-back can become an exchange of the p and wrk2
 * device buffers (OFL_FUSE_COPYBACK_SWAP: exact, because the sweep writes only
 * the interior and wrk2's device copy first receives p's boundary). Results
 * equal the unfused path's up to the residual's summation order; wrk2's device
 * content after a run is unspecified (it is scratch). Other genes, per-iteration
 * placement and batched runs ignore the setting. The fused residual sums in
 * FP64 only, so OFL_FUSE_RESIDUAL on a grid created with OFL_SUM_KAHAN_F32 is
 * refused (ENOTSUP) rather than reporting an FP64 sum as a compensated one.
 * EINVAL for unknown bits; ESTATE while the grid belongs to a batch. */
#define OFL_FUSE_RESIDUAL 1u
#define OFL_FUSE_COPYBACK_SWAP 2u
int ofl_set_fusion(ofl_grid *g, unsigned flags);

/* Per-array FP32 bias of the bfloat16-offset format (zeros for the other
 * formats), in coefficient order. */
int ofl_grid_coef_bias(const ofl_grid *g, float bias[12]);

/* ---- kernel tiles ------------------------------------------------------- */
#define OFL_TILE_NT_LOADS 1   /* non-temporal loads of the coefficient streams (sweep), of wrk2
                                 (copy-back) and of a batch residual's inputs; a single grid's
                                 residual always loads ordinarily, leaving p and wrk2 cached
                                 for the copy-back that follows */
#define OFL_TILE_NT_STORES 2  /* non-temporal stores of wrk2 (sweep) and p (copy-back); a single
                                 grid whose p takes 48 to 224 MiB stores p ordinarily in the
                                 copy-back, so that the next sweep finds it in the last-level cache */
#define OFL_TILE_PREFETCH 4   /* software-pipelined coefficient loads (next step during this one) */
#define OFL_TILE_MARCH_J 8    /* waves march along j (own a k-plane) instead of along k (own a j-row) */
#define OFL_TILE_XCD_REMAP 16 /* give each XCD one contiguous range of the sweep's tiles over the
                                 whole grid; by default each XCD takes one contiguous band of
                                 every k-chunk's tiles (when a k-chunk holds a multiple of 8;
                                 else tiles go round-robin), so all XCDs stream one window of
                                 HBM while j-neighbours share an L2 */

typedef struct ofl_tile {
    int vec;       /* consecutive i-points per lane: 1, 2 or 4 (a wave spans 64*vec points),
                      or 8 (single grids marching along k, row pitch a multiple of 8
                      elements: a wave spans two rows of 256 points, one per half-wave);
                      batches also accept 0: each grid gets the width that leaves the
                      fewest idle lanes on its rows (one batched launch for all widths) */
    int rows;      /* lines per work-group = waves per work-group: 1..8 (j-rows, or k-planes
                      with OFL_TILE_MARCH_J) */
    int kchunk;    /* steps each wave marches through (k-planes, or j-rows with
                      OFL_TILE_MARCH_J): 1..1024 */
    int flags;     /* OFL_TILE_* */
    int occupancy; /* 0..16. Single grid: at most this many sweep work-groups resident
                      per CU, 0 = as many as registers allow (the sweep launch reserves
                      LDS it does not use; EINVAL from the run if the device cannot hold
                      that reservation). Batched launch: resident work-groups per CU of
                      persistent kernels, 0 = one work-group per work item */
} ofl_tile;

/* Set / read the sweep tile of a grid. EINVAL for values outside the ranges.
 * Until a tile is set here or by ofl_grid_tune, the grid uses its default:
 * vec 4, 2 or 1 for more than 128, 64 or fewer interior points per row;
 * 4 rows; 2-plane chunks; non-temporal loads; non-temporal stores for FP32
 * coefficients, and for the bfloat16 formats while OFL_FUSE_COPYBACK_SWAP is
 * set (ofl_set_fusion re-derives the default); for FP32 coefficients at
 * vec 4, occupancy 3 and, unless OFL_FUSE_RESIDUAL is set,
 * OFL_TILE_PREFETCH; else occupancy 0. */
int ofl_set_tile(ofl_grid *g, const ofl_tile *tile);
int ofl_get_tile(const ofl_grid *g, ofl_tile *tile);

/* ---- statistics ----------------------------------------------------------- */
typedef struct ofl_stats {
    uint64_t h2d_count, d2h_count;  /* array transfers issued (scalars excluded) */
    uint64_t h2d_bytes, d2h_bytes;  /* their payload bytes */
    uint64_t gpu_nests[3];          /* nest executions on the GPU: S, R, C */
    uint64_t cpu_nests[3];          /* nest executions on the CPU: S, R, C */
    double kernel_ms[3];            /* summed GPU time of S, R, C (profiling on) */
    uint64_t timed_nests[3];        /* executions included in kernel_ms */
    uint64_t gpu_regions[3];        /* GPU region launches of S, R, C (one per nest at OFL_LEVEL_K) */
} ofl_stats;

/* Profiling on: each GPU nest is bracketed by HIP events on the grid's stream
 * and its time is added to kernel_ms at the next synchronisation. A nest split
 * into regions is bracketed as a whole; under the per-iteration placement it is
 * not timed, since its transfers sit between its launches. In fused runs the
 * copy-back exchange launches nothing and the residual sums of all iterations
 * but the last run inside the next sweep launch, so the residual is timed once
 * per run. */
int ofl_set_profiling(ofl_grid *g, int on);

/* Which nests profiling brackets (bit n: nest n, as in the offload mask;
 * default all three). Each bracket adds two event records between kernels,
 * so timing only the nest of interest disturbs the rest least. EINVAL for
 * bits above 2. */
int ofl_set_profiled_nests(ofl_grid *g, unsigned nests);
int ofl_get_stats(const ofl_grid *g, ofl_stats *out);
int ofl_reset_stats(ofl_grid *g);

/* ---- the transfer planner as a pure function ------------------------------ */
typedef struct ofl_xfer {
    int iter;   /* iteration index; -1 before the loop (data_enter), iters after it */
    int nest;   /* 0 S, 1 R, 2 C (nest index for ofl_plan_nests); -1 outside the nests */
    int when;   /* 0 before the nest, 1 after it */
    int array;  /* OFL_ARR_* */
    int dir;    /* 0 host->device, 1 device->host */
} ofl_xfer;

/* The transfers ofl_jacobi_run would issue for this mask and mode (Sec. 4.2.2
 * rules), without touching any data. host_valid/dev_valid (14 entries each,
 * 0/1, OFL_ARR_* order) give the state before the run and receive the state
 * after it; sync_host_at_end = 1 models a run outside a data region. Writes at
 * most cap entries to out (nullable when cap == 0) and the full count to
 * *count. EINVAL for bad mask/mode/iters; ENOMEM (count still set) when cap is
 * too small. */
int ofl_plan(unsigned mask, int xfer_mode, int iters, int sync_host_at_end, uint8_t host_valid[14],
             uint8_t dev_valid[14], ofl_xfer *out, int cap, int *count);

/* The planner over any program of loop nests (Sec. 4.2.2: transfers follow from
 * which side sets and which side references each variable). Each nest is
 * given by bit sets over array ids 0..narrays-1: the arrays it reads, the
 * arrays it writes, and the arrays it writes only in part while the rest
 * stays live (those must be whole on the writer's side first, so they move as
 * if read). live_after: arrays the CPU program references after the loop. The
 * gene `mask` has one bit per nest (1 = GPU). Otherwise as ofl_plan, which is
 * this function on the table ofl_program_vars returns. EINVAL for nnests
 * outside 1..OFL_MAX_NESTS, narrays outside 1..OFL_MAX_ARRAYS, bits beyond
 * narrays or nnests, or bad state/output arguments. */
#define OFL_MAX_NESTS 8
#define OFL_MAX_ARRAYS 32
typedef struct ofl_nest_vars {
    uint32_t reads;    /* bit a: the nest reads array a */
    uint32_t writes;   /* bit a: the nest writes array a */
    uint32_t partial;  /* bit a: it writes part of array a, the rest of which stays live */
} ofl_nest_vars;
int ofl_plan_nests(const ofl_nest_vars *nests, int nnests, int narrays, uint32_t live_after, unsigned mask,
                   int xfer_mode, int iters, int sync_host_at_end, uint8_t *host_valid, uint8_t *dev_valid,
                   ofl_xfer *out, int cap, int *count);

/* The library's program in that form: the nests S, R, C over the OFL_ARR_*
 * arrays, and the arrays referenced after the loop (p). EINVAL on NULL. */
int ofl_program_vars(ofl_nest_vars out[3], uint32_t *live_after);

/* ---- many independent grids in one launch sequence -------------------------
 * Not a step of the paper's method: the paper offloads one program run at a
 * time. A batch serves many independent instances of the offloaded program
 * (grids of uneven sizes) with the same gene (111, hoisted) in one graph
 * launch. Errors: a device error in a batched call makes the batch and every
 * grid in it unusable (OFL_EDEVICE from then on; destroy the batch, then the
 * grids); a device error in ofl_batch_create leaves the grids as they were. */
typedef struct ofl_batch ofl_batch;

/* Group n grids (all on one device, one coefficient format and sum mode) for
 * one batched run: every grid's S, R and C over all iterations run as
 * batched kernels over a work list of tiles sorted largest grid first,
 * captured once into a HIP graph and launched as one graph. The grids keep
 * ownership of their arrays; the batch borrows them and must be destroyed
 * first. tile may be NULL: the vector width per grid (vec 0), 1 line per
 * work-group, 2-plane chunks for FP32 coefficients and 4-plane ones for the
 * bfloat16 formats, non-temporal loads and stores; unfused bfloat16 batches
 * take vec 4 and 2 lines per work-group instead (ofl_batch_set_fusion
 * re-derives the default until a tile is set or searched). Unless the tile
 * has OFL_TILE_XCD_REMAP, each grid's sweep items are ordered so that every
 * XCD receives runs of consecutive lines (which share halo rows). A grid created
 * with a compact desc.row_align whose rows fill few of a wave's lanes runs in
 * packed rows: each wave covers 64 * vec consecutive points of a plane across
 * row ends. EINVAL for n < 1, NULL grids, mixed devices or formats. */
int ofl_batch_create(ofl_grid *const *grids, int n, const ofl_tile *tile, ofl_batch **out);
void ofl_batch_destroy(ofl_batch *b);
int ofl_batch_set_tile(ofl_batch *b, const ofl_tile *tile);
int ofl_batch_get_tile(const ofl_batch *b, ofl_tile *tile);

/* Fusion for the batched iterations (OFL_FUSE_* as for ofl_set_fusion): the
 * batched sweep also emits each grid's residual partials, and/or the copy-back
 * becomes an exchange of every grid's p and wrk2 buffers (odd iterations read
 * a second view table with the two exchanged; after a run of odd length the
 * grids keep the exchange). EINVAL for unknown bits; ENOTSUP for
 * OFL_FUSE_RESIDUAL on a batch of OFL_SUM_KAHAN_F32 grids (the fused residual
 * sums in FP64 only). */
int ofl_batch_set_fusion(ofl_batch *b, unsigned flags);

/* iters x (S, R, C) on the GPU for every grid of the batch, inside the
 * grids' data regions when open (else the grids' p are copied back at the
 * end). gosa_out (nullable) receives n residuals, one per grid. The first
 * call for a given iters/omega captures and instantiates the graph; later
 * calls replay it. */
int ofl_batch_run(ofl_batch *b, int iters, float omega, double *gosa_out);

/* ---- genetic-algorithm tile tuner (Sec. 4.2.2 search, over tile genes) ---- */
typedef struct ofl_ga_params {
    int population;     /* individuals per generation, >= 2 */
    int generations;    /* >= 1 */
    uint64_t seed;      /* random seed of the search */
    double crossover;   /* single-point crossover probability, 0..1 */
    double mutation;    /* per-bit mutation probability, 0..1 */
    int elite;          /* best individuals copied unchanged, >= 0 */
    int probe_iters;    /* Jacobi iterations per timing run, >= 1 */
    int repeats;        /* timing runs per individual (median taken), >= 1 */
    double tolerance;   /* max relative error vs the all-CPU nests on the check grid */
} ofl_ga_params;

typedef struct ofl_tune_result {
    ofl_tile best;
    double best_ms;     /* median time of probe_iters iterations with the best tile */
    int evaluated;      /* distinct genes measured */
    int rejected;       /* genes that could not be built or gave wrong results */
    int from_cache;     /* of the evaluated genes, those whose time came from the tune cache file */
} ofl_tune_result;

/* Search sweep tiles for one grid (or for a batch) with a GA: genes are bit
 * strings encoding an ofl_tile; a gene whose tile cannot be launched scores
 * zero, a gene whose result on a small check grid differs from the all-CPU
 * nests beyond the tolerance gets infinite time (Sec. 4.2.2), the rest are
 * timed with HIP events; roulette selection on 1/sqrt(time), single-point
 * crossover, per-bit mutation and elite copy make the next generation. The
 * best tile is also applied to the grid/batch. p is restored on return. */
int ofl_grid_tune(ofl_grid *g, const ofl_ga_params *ga, ofl_tune_result *out);
int ofl_batch_tune(ofl_batch *b, const ofl_ga_params *ga, ofl_tune_result *out);

/* Measurements kept across searches (checkpoint and resume of a tile search;
 * not a paper passage: the method measures every pattern, and this keeps
 * those measurements). With a path set, ofl_grid_tune and ofl_batch_tune read
 * the file's earlier measurements before searching and append every gene they
 * measure as soon as it is measured, one text line each:
 *   ofl-tune 1 <key> <gene in hex> <ms, inf (wrong result) or nan (not built)>
 * The key names what a gene's time depends on besides the gene: grid shapes,
 * coefficient format, summation mode, fusion, row alignment, probe_iters,
 * repeats, tolerance, the device (architecture and compute units) and a hash
 * of the library's sources. A gene found under the search's key is not
 * measured again (ofl_tune_result.from_cache counts them), so a stopped search
 * resumes where it stopped and a search with other GA parameters reuses what
 * was measured. Lines under other keys are kept and ignored. path NULL (the
 * default) keeps no file. Process-wide; the path is read when a tuner starts.
 * A file that cannot be opened for appending makes that tuner call fail
 * (EINVAL) before any measurement. EINVAL for a path holding a newline. */
int ofl_set_tune_cache(const char *path);

/* The GA of Sec. 4.2.2 over arbitrary bit genes with a caller-supplied
 * measurement: the initial population is random (seed_gene joins it), each
 * distinct gene is measured once by eval(gene, ctx), which returns its time
 * (> 0), +INFINITY when its result differs from the original program's, or NaN
 * when the gene cannot be built (both score zero); fitness is 1/sqrt(time);
 * roulette selection, single-point crossover, per-bit mutation and an
 * unchanged copy of the elite make each next generation. bits: 1..30. Runs on
 * the host only (no GPU needed unless eval uses one). EINVAL for bad bits,
 * parameters or NULL pointers. */
typedef double (*ofl_gene_eval)(uint32_t gene, void *ctx);
typedef struct ofl_ga_result {
    uint32_t best_gene;
    double best_time;   /* +INFINITY if no gene scored */
    int evaluated;      /* distinct genes measured */
    int rejected;       /* genes that were wrong or not buildable */
} ofl_ga_result;
int ofl_ga_search(int bits, const ofl_ga_params *ga, uint32_t seed_gene, ofl_gene_eval eval, void *ctx,
                  ofl_ga_result *out);

/* The paper's loop-offload search (Sec. 3.2.1, Sec. 4.2.2) on one grid: the
 * gene is the 3-bit offload mask plus one bit for the transfer placement
 * (bit 3: 1 = hoisted). Each gene runs iters iterations from the grid's current
 * p with nothing on the device, end to end (transfers included, host clock,
 * median of ga->repeats runs);
 * a result that differs from the all-CPU gene's (the original program) beyond
 * ga->tolerance gets infinite time. The best gene is applied to the grid and
 * p is restored. Needs a GPU for genes with GPU nests. ESTATE inside a data
 * region or a batch. */
typedef struct ofl_offload_result {
    unsigned mask;      /* best offload gene, bit = 1 -> GPU */
    int xfer_mode;      /* best placement */
    double best_ms;     /* its measured time */
    double cpu_ms;      /* the all-CPU gene's time */
    int evaluated, rejected;
} ofl_offload_result;
int ofl_grid_search_offload(ofl_grid *g, const ofl_ga_params *ga, int iters, float omega, ofl_offload_result *out);

/* The same search over the loop gene of ofl_set_loop_gene (Sec. 4.2.2: the
 * loops that fail the screen are left out, the rest make the gene), with the
 * given transfer placement. Each gene runs iters iterations from the grid's
 * current p with nothing on the device, timed end to end on the host clock
 * (median of ga->repeats runs);
 * genes that open the same regions share one measurement. A result that
 * differs from the all-CPU gene's beyond ga->tolerance gets infinite time, and
 * so does a gene with a run still going after time_limit_ms (<= 0: ten
 * times the all-CPU gene's time), which is stopped there. The best gene is applied to
 * the grid and p is restored. ESTATE inside a data region or a batch, or when
 * no gene reproduces the all-CPU result. */
typedef struct ofl_loop_search_result {
    uint32_t gene;      /* best loop gene */
    unsigned mask;      /* the regions it opens */
    int level[3];
    int gene_bits;      /* gene length: loops that passed the screen */
    double best_ms;     /* its measured time */
    double cpu_ms;      /* the all-CPU gene's time */
    int evaluated;      /* distinct genes scored */
    int patterns;       /* distinct region patterns measured */
    int rejected;       /* patterns whose result was wrong */
    int timed_out;      /* patterns stopped at the time limit */
} ofl_loop_search_result;
int ofl_grid_search_loops(ofl_grid *g, const ofl_ga_params *ga, int iters, float omega, int xfer_mode,
                          double time_limit_ms, ofl_loop_search_result *out);

/* ---- function-block offload (Sec. 3.2.2, Sec. 4.2.1) ----------------------
 * GPU routines that a recognised host function block (a call of a known
 * library routine) is replaced with; the Python front end's pattern table
 * maps numpy's matrix products onto ofl_gemm_f32. */

/* Matrix product C = A B of row-major FP32 matrices in device memory: A is
 * M x K with row stride lda >= K, B is K x N with ldb >= N, C is M x N with
 * ldc >= N (strides in elements). C must not overlap A or B. The library's
 * matrix-core kernel (FP32 products, FP32 accumulation) is queued on stream (a
 * hipStream_t; NULL: the default stream) and the call returns without
 * waiting. Nothing is read or written when M or N is 0; K = 0 sets C to 0.
 * EINVAL for negative sizes, M above 65535 * 128, short strides, or a NULL
 * pointer to an operand the product reads or writes; EDEVICE when the launch
 * fails. */
int ofl_gemm_f32(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
                 void *stream);

/* ---- measurement helper ---------------------------------------------------- */
/* Device-to-device copy of bytes (multiple of 16, 16-byte aligned pointers)
 * with the library's streaming copy kernel on the given stream (NULL = the
 * default stream): the rate of a 1:1 read + write stream. */
int ofl_device_copy(void *dst, const void *src, size_t bytes, void *stream);

/* The sweep's streaming pattern without the stencil, as a ceiling to compare
 * the sweep with: dst[t] = sum over the n32 FP32 sources src32[s][t] plus
 * sum over the n16 bfloat16 sources src16[s][t] (widened), for t < n. Every
 * array is a separate contiguous device array, read with non-temporal loads of
 * 4 elements per lane in linear order, dst written the same way; queued on
 * stream (NULL: the default stream). (n32, n16) must be (13, 0), the FP32
 * sweep's 13 reads and 1 write per point (56 bytes), or (1, 12), the bfloat16
 * sweep's (32 bytes); other counts give ENOTSUP. EINVAL for NULL pointers, n
 * not a multiple of 4, or sources/dst not aligned to their vector (16 bytes
 * for FP32, 8 for bfloat16). */
int ofl_device_stream(const float *const *src32, int n32, const uint16_t *const *src16, int n16, float *dst,
                      size_t n, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *ofl_last_error(void);

/* Library version string. */
const char *ofl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OFL_H */
