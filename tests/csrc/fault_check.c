/* Device-error paths of the C interface, on the stand-in HIP runtime
 * (hip_stand_in.cpp) with no-op kernel launchers: the device state exists
 * (blocks, streams, graphs, batch tables) but nothing runs on a GPU, so every
 * HIP call the library makes can be made to fail in turn.
 *
 * For each call n of a sequence of interface calls, a fresh handle runs the
 * sequence with the n-th HIP call failing. The sticky-error rule of ofl.h
 * must hold: once the device state of a handle exists, the first failing
 * interface call reports OFL_EDEVICE and so does every later call that would
 * touch the device; before it exists (no device, the first allocation
 * failing) the handle stays usable. Destroying the handles afterwards must
 * give back every allocation and token the stand-in handed out. Built with
 * address, leak and undefined-behaviour sanitizers by the test suite; exits 0
 * when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include "ofl.h"

void stand_in_fail_call(long n);
long stand_in_calls(void);
long stand_in_live(void);
long stand_in_alloc_calls(void);

#define CHECK(c)                                                                                       \
    do {                                                                                               \
        if (!(c)) {                                                                                    \
            fprintf(stderr, "FAIL %s:%d: %s (last error: %s)\n", __FILE__, __LINE__, #c,               \
                    ofl_last_error());                                                                 \
            return 1;                                                                                  \
        }                                                                                              \
    } while (0)

typedef struct {
    int I, J, K;
    float *arr[14];
} problem;

static void make(problem *pb, int I, int J, int K) {
    size_t n = (size_t)I * J * K;
    pb->I = I;
    pb->J = J;
    pb->K = K;
    for (int a = 0; a < 14; ++a) {
        pb->arr[a] = (float *)malloc(n * sizeof(float));
        for (size_t t = 0; t < n; ++t)
            pb->arr[a][t] = a == 3 ? 1.0f / 6.0f : (a < 3 || (a >= 7 && a <= 10) ? 1.0f : 0.25f);
    }
}

static void drop(problem *pb) {
    for (int a = 0; a < 14; ++a)
        free(pb->arr[a]);
}

static ofl_grid_desc desc_of(problem *pb, int fmt) {
    ofl_grid_desc d;
    memset(&d, 0, sizeof d);
    d.I = pb->I;
    d.J = pb->J;
    d.K = pb->K;
    d.coef_format = fmt;
    d.sum_mode = OFL_SUM_F64;
    d.p = pb->arr[12];
    d.wrk2 = pb->arr[13];
    for (int a = 0; a < 12; ++a)
        d.coef[a] = pb->arr[a];
    d.device = -1;
    return d;
}

/* One step of a grid sequence: 0 on success, else the status. */
static int grid_step(ofl_grid *g, int step) {
    static const int lev_mixed[3] = {OFL_LEVEL_J, OFL_LEVEL_I, OFL_LEVEL_K};
    ofl_tile t;
    double x;
    switch (step) {
    case 0: return ofl_jacobi_run(g, 3, 0.8f, &x);             /* graphed steady state */
    case 1: return ofl_residual(g, &x);
    case 2: return ofl_set_fusion(g, OFL_FUSE_RESIDUAL | OFL_FUSE_COPYBACK_SWAP);
    case 3: return ofl_jacobi_run(g, 3, 0.8f, &x);             /* fused, odd: buffers exchanged */
    case 4: return ofl_set_fusion(g, 0);
    case 5: return ofl_set_profiling(g, 1);
    case 6: return ofl_jacobi_run(g, 2, 0.8f, &x);             /* nest by nest, events */
    case 7: return ofl_set_regions(g, 7u, lev_mixed, OFL_XFER_PER_ITER);
    case 8: return ofl_jacobi_run(g, 1, 0.8f, &x);             /* regions, per-iteration copies */
    case 9: return ofl_set_offload_mask(g, 5u, OFL_XFER_HOISTED);
    case 10: return ofl_jacobi_run(g, 2, 0.8f, &x);            /* mixed gene, residual on the CPU */
    case 11: return ofl_set_offload_mask(g, OFL_MASK_ALL_GPU, OFL_XFER_HOISTED);
    case 12: return ofl_data_enter(g);
    case 13: return ofl_jacobi_run(g, 2, 0.8f, &x);
    case 14: return ofl_update_host(g);
    case 15: return ofl_data_exit(g);
    case 16:
        if (ofl_get_tile(g, &t) != OFL_OK)
            return -100;
        t.kchunk = 3;
        return ofl_set_tile(g, &t);
    case 17: return ofl_reset_stats(g);
    default: return ofl_jacobi_run(g, 1, 0.8f, &x);
    }
}
#define GRID_STEPS 19

/* Every call on an unusable grid that would touch its state reports OFL_EDEVICE. */
static int grid_refuses(ofl_grid *g) {
    double x;
    int lev[3] = {0, 0, 0};
    ofl_tile t = {4, 4, 2, 1, 0};
    CHECK(ofl_jacobi_run(g, 1, 0.8f, &x) == OFL_EDEVICE);
    CHECK(ofl_residual(g, &x) == OFL_EDEVICE);
    CHECK(ofl_jacobi_run_static(g, 1, 0.8f, &x) == OFL_EDEVICE);
    CHECK(ofl_set_offload_mask(g, 0u, OFL_XFER_HOISTED) == OFL_EDEVICE);
    CHECK(ofl_set_regions(g, 7u, lev, OFL_XFER_HOISTED) == OFL_EDEVICE);
    CHECK(ofl_set_loop_gene(g, 1u, OFL_XFER_HOISTED) == OFL_EDEVICE);
    CHECK(ofl_data_enter(g) == OFL_EDEVICE);
    CHECK(ofl_update_host(g) == OFL_EDEVICE);
    CHECK(ofl_data_exit(g) == OFL_EDEVICE);
    CHECK(ofl_set_fusion(g, 0u) == OFL_EDEVICE);
    CHECK(ofl_set_tile(g, &t) == OFL_EDEVICE);
    CHECK(ofl_set_profiling(g, 0) == OFL_EDEVICE);
    CHECK(ofl_reset_stats(g) == OFL_EDEVICE);
    CHECK(strstr(ofl_last_error(), "unusable") != NULL);
    ofl_batch *b = NULL;
    CHECK(ofl_batch_create(&g, 1, NULL, &b) == OFL_EDEVICE && b == NULL);
    return 0;
}

/* The grid sequence with its n-th HIP call failing (n = 0: none); *calls
 * receives the HIP calls the sequence made, *failed whether a step failed. */
static int grid_case(long n, long *calls, int *failed) {
    problem pb;
    make(&pb, 37, 9, 7);
    const long live0 = stand_in_live();
    ofl_grid_desc d = desc_of(&pb, n % 2 ? OFL_COEF_BF16_OFFSET : OFL_COEF_F32);
    ofl_grid *g = NULL;
    CHECK(ofl_grid_create(&d, &g) == OFL_OK);
    double x;
    CHECK(ofl_jacobi_run(g, 2, 0.8f, &x) == OFL_OK); /* the device state exists from here on */
    stand_in_fail_call(n);
    int first_bad = -1;
    for (int s = 0; s < GRID_STEPS; ++s) {
        const int rc = grid_step(g, s);
        if (first_bad < 0 && rc != OFL_OK) {
            CHECK(rc == OFL_EDEVICE);
            first_bad = s;
        } else if (first_bad >= 0) {
            /* calls that only record a setting still refuse: the handle is unusable */
            CHECK(rc == OFL_EDEVICE);
        }
    }
    *calls = stand_in_calls();
    stand_in_fail_call(0);
    *failed = first_bad >= 0;
    if (first_bad >= 0 && grid_refuses(g) != 0)
        return 1;
    ofl_stats st;
    CHECK(ofl_get_stats(g, &st) == OFL_OK); /* reading the statistics stays valid */
    ofl_grid_destroy(g);
    CHECK(stand_in_live() == live0);
    drop(&pb);
    return 0;
}

/* First GPU use with the n-th HIP call failing: before the device state
 * exists the handle stays usable, after it the error is sticky. */
static int first_use_case(long n, long *calls, int *sticky) {
    problem pb;
    make(&pb, 21, 6, 5);
    const long live0 = stand_in_live();
    ofl_grid_desc d = desc_of(&pb, OFL_COEF_F32);
    ofl_grid *g = NULL;
    CHECK(ofl_grid_create(&d, &g) == OFL_OK);
    double x;
    stand_in_fail_call(n);
    const int rc = ofl_jacobi_run(g, 2, 0.8f, &x);
    *calls = stand_in_calls();
    stand_in_fail_call(0);
    CHECK(rc == OFL_OK || rc == OFL_EDEVICE || rc == OFL_ENOMEM);
    const int rc2 = ofl_jacobi_run(g, 2, 0.8f, &x);
    *sticky = rc2 == OFL_EDEVICE;
    CHECK(rc2 == OFL_OK || (rc == OFL_EDEVICE && rc2 == OFL_EDEVICE));
    if (rc2 == OFL_OK) {
        /* a usable handle also runs an all-CPU gene */
        CHECK(ofl_set_offload_mask(g, OFL_MASK_ALL_CPU, OFL_XFER_HOISTED) == OFL_OK);
        CHECK(ofl_jacobi_run(g, 1, 0.8f, &x) == OFL_OK);
    }
    ofl_grid_destroy(g);
    CHECK(stand_in_live() == live0);
    drop(&pb);
    return 0;
}

static int batch_step(ofl_batch *b, int step, double *gosa) {
    ofl_tile t;
    switch (step) {
    case 0: return ofl_batch_run(b, 3, 0.8f, gosa);
    case 1: return ofl_batch_run(b, 3, 0.8f, gosa);          /* graph replay */
    case 2: return ofl_batch_set_fusion(b, OFL_FUSE_RESIDUAL | OFL_FUSE_COPYBACK_SWAP);
    case 3: return ofl_batch_run(b, 3, 0.8f, gosa);          /* odd: view tables refreshed */
    case 4:
        if (ofl_batch_get_tile(b, &t) != OFL_OK)
            return -100;
        t.rows = 2;
        return ofl_batch_set_tile(b, &t);                    /* tables rebuilt */
    default: return ofl_batch_run(b, 2, 0.8f, gosa);
    }
}
#define BATCH_STEPS 6

/* A batch of three grids (one in compact rows) with its n-th HIP call failing,
 * from batch creation on (n = 0: none). */
static int batch_case(long n, long *calls, int *failed) {
    problem pb[3];
    make(&pb[0], 37, 9, 7);
    make(&pb[1], 70, 5, 6);
    make(&pb[2], 11, 13, 5);
    const long live0 = stand_in_live();
    ofl_grid *g[3];
    for (int t = 0; t < 3; ++t) {
        ofl_grid_desc d = desc_of(&pb[t], OFL_COEF_F32);
        d.row_align = t == 2 ? 4 : 0;
        CHECK(ofl_grid_create(&d, &g[t]) == OFL_OK);
        double x;
        CHECK(ofl_jacobi_run(g[t], 1, 0.8f, &x) == OFL_OK);
    }
    stand_in_fail_call(n);
    ofl_batch *b = NULL;
    const int rc = ofl_batch_create(g, 3, NULL, &b);
    int first_bad = -1;
    double gosa[3];
    if (rc != OFL_OK) {
        CHECK(rc == OFL_EDEVICE && b == NULL);
        first_bad = 0;
    } else {
        for (int s = 0; s < BATCH_STEPS; ++s) {
            const int r = batch_step(b, s, gosa);
            if (first_bad < 0 && r != OFL_OK) {
                CHECK(r == OFL_EDEVICE);
                first_bad = s + 1;
            } else if (first_bad >= 0) {
                CHECK(r == OFL_EDEVICE);
            }
        }
    }
    *calls = stand_in_calls();
    stand_in_fail_call(0);
    *failed = first_bad >= 0;
    if (b && first_bad >= 0) {
        /* the batch and its grids are unusable */
        CHECK(ofl_batch_run(b, 1, 0.8f, gosa) == OFL_EDEVICE);
        CHECK(ofl_batch_set_fusion(b, 0u) == OFL_EDEVICE);
        for (int t = 0; t < 3; ++t)
            if (grid_refuses(g[t]) != 0)
                return 1;
    }
    if (b)
        ofl_batch_destroy(b);
    for (int t = 0; t < 3; ++t)
        ofl_grid_destroy(g[t]);
    CHECK(stand_in_live() == live0);
    for (int t = 0; t < 3; ++t)
        drop(&pb[t]);
    return 0;
}

/* ofl_jacobi_run_static: its preconditions are refused before any work, and
 * on a resident fused grid it makes no HIP call that allocates or releases
 * (memory, streams, events, graphs), where ofl_jacobi_run takes its partials. */
static int static_case(void) {
    problem pb;
    make(&pb, 37, 9, 7);
    const long live0 = stand_in_live();
    ofl_grid_desc d = desc_of(&pb, OFL_COEF_F32);
    ofl_grid *g = NULL;
    CHECK(ofl_grid_create(&d, &g) == OFL_OK);
    double x = 0.0;
    CHECK(ofl_jacobi_run_static(g, 2, 0.8f, &x) == OFL_ESTATE); /* no device state */
    CHECK(ofl_jacobi_run_static(g, -1, 0.8f, &x) == OFL_EINVAL);
    CHECK(ofl_jacobi_run_static(g, 2, 0.0f, &x) == OFL_EINVAL);
    CHECK(ofl_set_fusion(g, OFL_FUSE_RESIDUAL) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 2, 0.8f, &x) == OFL_ESTATE); /* device state, no data region */
    CHECK(ofl_data_enter(g) == OFL_OK);
    long a0 = stand_in_alloc_calls();
    CHECK(ofl_jacobi_run_static(g, 3, 0.8f, &x) == OFL_OK);
    CHECK(ofl_set_fusion(g, OFL_FUSE_RESIDUAL | OFL_FUSE_COPYBACK_SWAP) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 3, 0.8f, &x) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 0, 0.8f, &x) == OFL_OK && isnan(x));
    CHECK(stand_in_alloc_calls() == a0);
    CHECK(ofl_jacobi_run(g, 1, 0.8f, &x) == OFL_OK); /* the allocating form takes its partials */
    CHECK(stand_in_alloc_calls() > a0);
    a0 = stand_in_alloc_calls();
    CHECK(ofl_jacobi_run_static(g, 2, 0.8f, &x) == OFL_OK);
    CHECK(stand_in_alloc_calls() == a0);
    CHECK(ofl_set_fusion(g, OFL_FUSE_COPYBACK_SWAP) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 1, 0.8f, &x) == OFL_ENOTSUP); /* no fused residual */
    CHECK(ofl_set_fusion(g, OFL_FUSE_RESIDUAL) == OFL_OK);
    CHECK(ofl_set_profiling(g, 1) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 1, 0.8f, &x) == OFL_ENOTSUP); /* events would be created */
    CHECK(ofl_set_profiling(g, 0) == OFL_OK);
    CHECK(ofl_set_offload_mask(g, 5u, OFL_XFER_HOISTED) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 1, 0.8f, &x) == OFL_ENOTSUP); /* not gene 111 */
    CHECK(ofl_set_offload_mask(g, OFL_MASK_ALL_GPU, OFL_XFER_PER_ITER) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 1, 0.8f, &x) == OFL_ENOTSUP); /* per-iteration placement */
    CHECK(ofl_set_offload_mask(g, OFL_MASK_ALL_GPU, OFL_XFER_HOISTED) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 1, 0.8f, &x) == OFL_OK);
    CHECK(ofl_data_exit(g) == OFL_OK);
    CHECK(ofl_jacobi_run_static(g, 1, 0.8f, &x) == OFL_ESTATE); /* region closed */
    ofl_grid_destroy(g);
    CHECK(stand_in_live() == live0);
    drop(&pb);
    return 0;
}

/* The tile tuner's measurement file on the stand-in runtime: no kernel runs,
 * so every gene's check fails and is recorded as a wrong result (inf), one
 * line per gene; a repeated search reads them all back and appends nothing;
 * an unwritable path is refused before any measurement. */
static long count_lines(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f)
        return -1;
    long n = 0;
    int c;
    while ((c = fgetc(f)) != EOF)
        n += c == '\n';
    fclose(f);
    return n;
}

static int cache_case(void) {
    char path[512];
    const char *tmp = getenv("TMPDIR");
    snprintf(path, sizeof path, "%s/ofl_tune_cache_%ld.txt", tmp && *tmp ? tmp : "/tmp", (long)getpid());
    remove(path);
    problem pb;
    make(&pb, 37, 9, 7);
    ofl_grid_desc d = desc_of(&pb, OFL_COEF_F32);
    ofl_grid *g = NULL;
    CHECK(ofl_grid_create(&d, &g) == OFL_OK);
    ofl_ga_params ga;
    memset(&ga, 0, sizeof ga);
    ga.population = 4;
    ga.generations = 2;
    ga.seed = 5;
    ga.crossover = 0.9;
    ga.mutation = 0.05;
    ga.elite = 1;
    ga.probe_iters = 1;
    ga.repeats = 1;
    ga.tolerance = 1e-5;
    ofl_tune_result r;
    CHECK(ofl_set_tune_cache(path) == OFL_OK);
    CHECK(ofl_grid_tune(g, &ga, &r) == OFL_ESTATE); /* no gene gives a right result without kernels */
    const long n1 = count_lines(path);
    CHECK(n1 > 0);
    CHECK(ofl_grid_tune(g, &ga, &r) == OFL_ESTATE);
    CHECK(count_lines(path) == n1); /* every gene read back, none measured */
    ga.seed = 6;
    CHECK(ofl_grid_tune(g, &ga, &r) == OFL_ESTATE);
    CHECK(count_lines(path) >= n1);
    char bad[600];
    snprintf(bad, sizeof bad, "%s.missing-dir/x.txt", path);
    CHECK(ofl_set_tune_cache(bad) == OFL_OK);
    CHECK(ofl_grid_tune(g, &ga, &r) == OFL_EINVAL);
    CHECK(strstr(ofl_last_error(), "tune cache") != NULL);
    CHECK(ofl_set_tune_cache(NULL) == OFL_OK);
    CHECK(ofl_set_tune_cache("a\nb") == OFL_EINVAL);
    ofl_grid_destroy(g);
    drop(&pb);
    remove(path);
    return 0;
}

int main(void) {
    long calls = 0, total = 0;
    int failed = 0, sticky = 0;

    /* the entry point that allocates nothing */
    CHECK(static_case() == 0);
    printf("static-scratch run: no allocating HIP call\n");
    CHECK(cache_case() == 0);
    printf("tune cache: written, read back, refused when unwritable\n");

    /* grids whose device state exists */
    CHECK(grid_case(0, &total, &failed) == 0 && !failed && total > 40);
    int hits = 0;
    for (long n = 1; n <= total; ++n) {
        if (grid_case(n, &calls, &failed) != 0) {
            fprintf(stderr, "grid case with HIP call %ld failing\n", n);
            return 1;
        }
        hits += failed;
    }
    /* a failing call is swallowed only where the library ignores the status on purpose */
    CHECK(hits > total / 2);
    printf("grid sequence: %ld HIP calls, %d of them fail an interface call\n", total, hits);

    /* first GPU use */
    CHECK(first_use_case(0, &total, &sticky) == 0 && !sticky);
    int nonsticky = 0, stickies = 0;
    for (long n = 1; n <= total; ++n) {
        if (first_use_case(n, &calls, &sticky) != 0) {
            fprintf(stderr, "first-use case with HIP call %ld failing\n", n);
            return 1;
        }
        if (n == 1)
            CHECK(!sticky); /* no device found: the handle stays usable */
        stickies += sticky;
        nonsticky += !sticky;
    }
    CHECK(stickies > 0 && nonsticky > 1);
    printf("first use: %ld HIP calls, %d sticky failures, %d before the device state\n", total, stickies, nonsticky);

    /* batches */
    CHECK(batch_case(0, &total, &failed) == 0 && !failed && total > 20);
    hits = 0;
    for (long n = 1; n <= total; ++n) {
        if (batch_case(n, &calls, &failed) != 0) {
            fprintf(stderr, "batch case with HIP call %ld failing\n", n);
            return 1;
        }
        hits += failed;
    }
    CHECK(hits > total / 2);
    printf("batch sequence: %ld HIP calls, %d of them fail an interface call\n", total, hits);
    CHECK(stand_in_live() == 0);
    printf("device-error paths ok\n");
    return 0;
}
