/* Drives every host-side path of the C interface (no GPU needed): all-CPU
 * gene runs in every storage format, residuals, data regions, the planner,
 * argument checks, statistics, tiles, fusion flags and the GA search. Built
 * with address and undefined-behaviour sanitizers by the test suite. Exits 0
 * when every check holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ofl.h"

#define CHECK(c)                                                                                 \
    do {                                                                                         \
        if (!(c)) {                                                                              \
            fprintf(stderr, "FAIL %s:%d: %s (last error: %s)\n", __FILE__, __LINE__, #c,         \
                    ofl_last_error());                                                           \
            return 1;                                                                            \
        }                                                                                        \
    } while (0)

static uint64_t rng = 88172645463325252ull;
static double uni(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * 0x1.0p-53;
}

typedef struct {
    int I, J, K;
    float *arr[14];
} problem;

static void make(problem *pb, int I, int J, int K) {
    size_t n = (size_t)I * J * K;
    pb->I = I;
    pb->J = J;
    pb->K = K;
    for (int a = 0; a < 14; ++a)
        pb->arr[a] = (float *)calloc(n, sizeof(float));
    for (size_t t = 0; t < n; ++t) {
        for (int d = 0; d < 3; ++d)
            pb->arr[d][t] = (float)(1.0 + 0.1 * (uni() - 0.5));
        pb->arr[3][t] = (float)(1.0 / (2.0 * (pb->arr[0][t] + pb->arr[1][t] + pb->arr[2][t])));
        for (int d = 4; d < 7; ++d)
            pb->arr[d][t] = (float)(0.02 * (uni() - 0.5));
        for (int d = 7; d < 10; ++d)
            pb->arr[d][t] = 1.0f;
        pb->arr[11][t] = (float)(0.2 * (uni() - 0.5));
        pb->arr[12][t] = (float)uni();
    }
    for (int k = 1; k < K - 1; ++k)
        for (int j = 1; j < J - 1; ++j)
            for (int i = 1; i < I - 1; ++i)
                pb->arr[10][i + (size_t)I * (j + (size_t)J * k)] = 1.0f;
}

static void drop(problem *pb) {
    for (int a = 0; a < 14; ++a)
        free(pb->arr[a]);
}

static ofl_grid_desc desc_of(problem *pb, int fmt, int sum) {
    ofl_grid_desc d;
    memset(&d, 0, sizeof d);
    d.I = pb->I;
    d.J = pb->J;
    d.K = pb->K;
    d.coef_format = fmt;
    d.sum_mode = sum;
    d.p = pb->arr[12];
    d.wrk2 = pb->arr[13];
    for (int a = 0; a < 12; ++a)
        d.coef[a] = pb->arr[a];
    d.device = -1;
    return d;
}

static double ga_eval(uint32_t gene, void *ctx) {
    uint32_t target = *(uint32_t *)ctx;
    if (gene & 0x80u)
        return NAN; /* not buildable */
    return 1.0 + __builtin_popcount((gene ^ target) & 0x7fu);
}

static int run_formats(int I, int J, int K) {
    for (int fmt = 0; fmt <= 2; ++fmt) {
        problem pb;
        make(&pb, I, J, K);
        size_t n = (size_t)I * J * K;
        float *p0 = (float *)malloc(n * sizeof(float));
        memcpy(p0, pb.arr[12], n * sizeof(float));
        ofl_grid_desc d = desc_of(&pb, fmt, fmt == 2 ? OFL_SUM_KAHAN_F32 : OFL_SUM_F64);
        ofl_grid *g = NULL;
        CHECK(ofl_grid_create(&d, &g) == OFL_OK && g);
        CHECK(ofl_set_offload_mask(g, OFL_MASK_ALL_CPU, OFL_XFER_HOISTED) == OFL_OK);
        double gosa = -1.0;
        CHECK(ofl_jacobi_run(g, 0, 0.8f, &gosa) == OFL_OK && isnan(gosa));
        CHECK(ofl_jacobi_run(g, 4, 0.8f, &gosa) == OFL_OK && isfinite(gosa) && gosa >= 0.0);
        double r = -1.0;
        CHECK(ofl_residual(g, &r) == OFL_OK && isfinite(r));
        /* the boundary layer never changes */
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < J; ++j)
                for (int i = 0; i < I; ++i)
                    if (i == 0 || j == 0 || k == 0 || i == I - 1 || j == J - 1 || k == K - 1) {
                        size_t t = i + (size_t)I * (j + (size_t)J * k);
                        CHECK(pb.arr[12][t] == p0[t]);
                    }
        /* a GPU gene on a host without a GPU reports a device error, the handle stays usable */
        CHECK(ofl_set_offload_mask(g, OFL_MASK_ALL_GPU, OFL_XFER_HOISTED) == OFL_OK);
        CHECK(ofl_jacobi_run(g, 1, 0.8f, &gosa) == OFL_EDEVICE);
        CHECK(ofl_set_offload_mask(g, OFL_MASK_ALL_CPU, OFL_XFER_PER_ITER) == OFL_OK);
        CHECK(ofl_jacobi_run(g, 2, 0.8f, &gosa) == OFL_OK);
        CHECK(ofl_data_enter(g) == OFL_OK && ofl_data_enter(g) == OFL_ESTATE);
        CHECK(ofl_jacobi_run(g, 1, 0.8f, NULL) == OFL_OK);
        CHECK(ofl_update_host(g) == OFL_OK && ofl_data_exit(g) == OFL_OK && ofl_data_exit(g) == OFL_ESTATE);
        ofl_stats st; /* S and R ran 4+1+2+1 times (ofl_residual runs S and R without C), C 4+2+1 */
        CHECK(ofl_get_stats(g, &st) == OFL_OK && st.cpu_nests[0] == 8 && st.cpu_nests[1] == 8 && st.cpu_nests[2] == 7 && st.gpu_nests[0] == 0 && st.h2d_count == 0);
        CHECK(ofl_reset_stats(g) == OFL_OK && ofl_get_stats(g, &st) == OFL_OK && st.cpu_nests[0] == 0);
        float bias[12];
        CHECK(ofl_grid_coef_bias(g, bias) == OFL_OK);
        if (fmt != OFL_COEF_BF16_OFFSET)
            for (int a = 0; a < 12; ++a)
                CHECK(bias[a] == 0.0f);
        ofl_tile t;
        CHECK(ofl_get_tile(g, &t) == OFL_OK);
        t.kchunk = 5;
        t.flags = OFL_TILE_MARCH_J | OFL_TILE_XCD_REMAP;
        CHECK(ofl_set_tile(g, &t) == OFL_OK);
        t.vec = 3;
        CHECK(ofl_set_tile(g, &t) == OFL_EINVAL);
        /* the fused residual sums in FP64 only: refused where the grid asks for compensated FP32 */
        CHECK(ofl_set_fusion(g, OFL_FUSE_RESIDUAL | OFL_FUSE_COPYBACK_SWAP) == (fmt == 2 ? OFL_ENOTSUP : OFL_OK));
        CHECK(ofl_set_fusion(g, OFL_FUSE_COPYBACK_SWAP) == OFL_OK);
        CHECK(ofl_set_fusion(g, 8u) == OFL_EINVAL);
        CHECK(ofl_jacobi_run(g, -1, 0.8f, &gosa) == OFL_EINVAL);
        CHECK(ofl_jacobi_run(g, 1, 0.0f, &gosa) == OFL_EINVAL);
        CHECK(ofl_jacobi_run(g, 1, NAN, &gosa) == OFL_EINVAL);
        CHECK(ofl_set_offload_mask(g, 8u, OFL_XFER_HOISTED) == OFL_EINVAL);
        CHECK(ofl_set_offload_mask(g, 1u, 7) == OFL_EINVAL);
        ofl_batch *b = NULL;
        CHECK(ofl_batch_create(&g, 1, NULL, &b) != OFL_OK && b == NULL);
        ofl_grid_destroy(g);
        free(p0);
        drop(&pb);
    }
    return 0;
}

int main(void) {
    if (run_formats(3, 3, 3) || run_formats(17, 9, 12) || run_formats(33, 20, 17) || run_formats(4, 7, 3))
        return 1;

    /* argument checks at creation */
    problem pb;
    make(&pb, 5, 4, 3);
    ofl_grid_desc d = desc_of(&pb, 0, 0);
    ofl_grid *g = NULL;
    CHECK(ofl_grid_create(NULL, &g) == OFL_EINVAL);
    d.I = 2;
    CHECK(ofl_grid_create(&d, &g) == OFL_EINVAL);
    d.I = 5;
    d.coef[4] = NULL;
    CHECK(ofl_grid_create(&d, &g) == OFL_EINVAL && strlen(ofl_last_error()) > 0);
    d.coef[4] = pb.arr[4];
    d.coef_format = 9;
    CHECK(ofl_grid_create(&d, &g) == OFL_EINVAL);
    d.coef_format = 0;
    {
        /* compact rows: valid alignments create a handle, others are refused */
        static const int bad[] = {1, 2, 3, 5, 12, 64, -4};
        for (unsigned t = 0; t < sizeof bad / sizeof bad[0]; ++t) {
            d.row_align = bad[t];
            CHECK(ofl_grid_create(&d, &g) == OFL_EINVAL && strstr(ofl_last_error(), "row_align") != NULL);
        }
        static const int good[] = {0, 4, 8, 16, 32};
        for (unsigned t = 0; t < sizeof good / sizeof good[0]; ++t) {
            d.row_align = good[t];
            CHECK(ofl_grid_create(&d, &g) == OFL_OK && g);
            ofl_grid_destroy(g);
            g = NULL;
        }
        d.row_align = 0;
    }
    drop(&pb);
    {
        /* an all-CPU run does not depend on the row alignment */
        problem pa, pc;
        make(&pa, 13, 9, 7);
        make(&pc, 13, 9, 7);
        for (int a = 0; a < 14; ++a) /* the same problem twice */
            memcpy(pc.arr[a], pa.arr[a], sizeof(float) * 13 * 9 * 7);
        ofl_grid_desc da = desc_of(&pa, 0, 0), dc = desc_of(&pc, 0, 0);
        dc.row_align = 4;
        ofl_grid *ga = NULL, *gc = NULL;
        CHECK(ofl_grid_create(&da, &ga) == OFL_OK && ofl_grid_create(&dc, &gc) == OFL_OK);
        CHECK(ofl_set_offload_mask(ga, OFL_MASK_ALL_CPU, OFL_XFER_HOISTED) == OFL_OK);
        CHECK(ofl_set_offload_mask(gc, OFL_MASK_ALL_CPU, OFL_XFER_HOISTED) == OFL_OK);
        double xa = 0, xc = 1;
        CHECK(ofl_jacobi_run(ga, 3, 0.8f, &xa) == OFL_OK && ofl_jacobi_run(gc, 3, 0.8f, &xc) == OFL_OK && xa == xc);
        CHECK(memcmp(pa.arr[12], pc.arr[12], sizeof(float) * 13 * 9 * 7) == 0);
        ofl_grid_destroy(ga);
        ofl_grid_destroy(gc);
        drop(&pa);
        drop(&pc);
    }
    size_t bytes = 0;
    CHECK(ofl_grid_device_bytes(257, 257, 513, OFL_COEF_F32, 0, &bytes) == OFL_OK && bytes > 14ull * 257 * 257 * 513 * 4);
    CHECK(ofl_grid_device_bytes(2, 3, 3, OFL_COEF_F32, 0, &bytes) == OFL_EINVAL);

    /* the planner, every gene and placement, with a too-small output */
    for (unsigned mask = 0; mask < 8; ++mask)
        for (int mode = 0; mode < 2; ++mode) {
            uint8_t hv[14], dv[14];
            memset(hv, 1, sizeof hv);
            memset(dv, 0, sizeof dv);
            int count = -1;
            int rc = ofl_plan(mask, mode, 5, 1, hv, dv, NULL, 0, &count);
            CHECK((rc == OFL_OK && count == 0) || (rc == OFL_ENOMEM && count > 0));
            ofl_xfer *xs = (ofl_xfer *)malloc(sizeof(ofl_xfer) * (size_t)(count + 1));
            memset(hv, 1, sizeof hv);
            memset(dv, 0, sizeof dv);
            int count2 = -1;
            CHECK(ofl_plan(mask, mode, 5, 1, hv, dv, xs, count, &count2) == OFL_OK && count2 == count);
            CHECK(hv[OFL_ARR_P] == 1);
            free(xs);
        }
    {
        uint8_t hv[14] = {0}, dv[14] = {0};
        int count;
        CHECK(ofl_plan(7, 1, 1, 1, hv, dv, NULL, 0, &count) == OFL_EINVAL);
    }

    /* the planner over a caller's program table equals ofl_plan on the library's own */
    {
        ofl_nest_vars nv[3];
        uint32_t live = 0;
        CHECK(ofl_program_vars(nv, &live) == OFL_OK && live == (1u << OFL_ARR_P));
        for (unsigned mask = 0; mask < 8; ++mask)
            for (int mode = 0; mode < 2; ++mode) {
                ofl_xfer a[256], b[256];
                uint8_t h1[14], d1[14], h2[32], d2[32];
                memset(h1, 1, sizeof h1);
                memset(d1, 0, sizeof d1);
                memset(h2, 1, sizeof h2);
                memset(d2, 0, sizeof d2);
                int ca = -1, cb = -2;
                CHECK(ofl_plan(mask, mode, 4, 1, h1, d1, a, 256, &ca) == OFL_OK);
                CHECK(ofl_plan_nests(nv, 3, 14, live, mask, mode, 4, 1, h2, d2, b, 256, &cb) == OFL_OK);
                CHECK(ca == cb && memcmp(a, b, sizeof(ofl_xfer) * (size_t)ca) == 0);
                CHECK(memcmp(h1, h2, 14) == 0 && memcmp(d1, d2, 14) == 0);
            }
        uint8_t h[32], d[32];
        int c;
        memset(h, 1, sizeof h);
        memset(d, 0, sizeof d);
        CHECK(ofl_plan_nests(nv, 0, 14, live, 0u, 1, 1, 1, h, d, NULL, 0, &c) == OFL_EINVAL);
        CHECK(ofl_plan_nests(nv, 3, 33, live, 0u, 1, 1, 1, h, d, NULL, 0, &c) == OFL_EINVAL);
        CHECK(ofl_plan_nests(nv, 3, 12, live, 0u, 1, 1, 1, h, d, NULL, 0, &c) == OFL_EINVAL);
        CHECK(ofl_plan_nests(nv, 3, 14, live, 8u, 1, 1, 1, h, d, NULL, 0, &c) == OFL_EINVAL);
        ofl_nest_vars bad = {1u, 0u, 2u};
        CHECK(ofl_plan_nests(&bad, 1, 4, 0u, 1u, 1, 1, 1, h, d, NULL, 0, &c) == OFL_EINVAL);
        ofl_nest_vars wide = {0xffffffffu, 1u, 0u};
        CHECK(ofl_plan_nests(&wide, 1, 32, 1u, 1u, 0, 2, 1, h, d, NULL, 0, &c) == OFL_ENOMEM && c == 66);
    }

    /* the loop table, every loop gene, region settings */
    {
        problem q;
        make(&q, 9, 7, 6);
        ofl_grid_desc dq = desc_of(&q, 0, 0);
        ofl_grid *gq = NULL;
        CHECK(ofl_grid_create(&dq, &gq) == OFL_OK);
        ofl_loop_info t[OFL_NLOOPS];
        CHECK(ofl_loop_table(gq, t) == OFL_OK && t[0].parallel == 0 && t[0].nest == -1);
        for (int l = 1; l < OFL_NLOOPS; ++l)
            CHECK(t[l].parallel == 1 && t[l].nest == (l - 1) / 3 && t[l].level == (l - 1) % 3);
        for (uint32_t gene = 0; gene < 512; ++gene) {
            unsigned mask = 99;
            int lev[3] = {-7, -7, -7}, mode = -7;
            CHECK(ofl_set_loop_gene(gq, gene, OFL_XFER_PER_ITER) == OFL_OK);
            CHECK(ofl_get_regions(gq, &mask, lev, &mode) == OFL_OK && mode == OFL_XFER_PER_ITER);
            for (int n = 0; n < 3; ++n) {
                unsigned bits = (gene >> (3 * n)) & 7u;
                CHECK(((mask >> n) & 1u) == (bits != 0));
                if (bits)
                    CHECK(lev[n] == __builtin_ctz(bits));
            }
        }
        CHECK(ofl_set_loop_gene(gq, 512u, OFL_XFER_HOISTED) == OFL_EINVAL);
        int lv[3] = {2, 1, 2};
        CHECK(ofl_set_regions(gq, 0u, lv, OFL_XFER_HOISTED) == OFL_OK);
        double gs = 0.0;
        CHECK(ofl_jacobi_run(gq, 2, 0.8f, &gs) == OFL_OK && isfinite(gs));
        lv[1] = 3;
        CHECK(ofl_set_regions(gq, 7u, lv, OFL_XFER_HOISTED) == OFL_EINVAL);
        CHECK(ofl_set_regions(gq, 7u, NULL, OFL_XFER_HOISTED) == OFL_EINVAL);
        CHECK(ofl_loop_table(NULL, t) == OFL_EINVAL);
        ofl_grid_destroy(gq);
        drop(&q);
    }

    /* matrix product: argument checks and empty products need no device */
    CHECK(ofl_gemm_f32(-1, 1, 1, NULL, 1, NULL, 1, NULL, 1, NULL) == OFL_EINVAL);
    CHECK(ofl_gemm_f32(2, 2, 2, NULL, 1, NULL, 2, NULL, 2, NULL) == OFL_EINVAL);
    CHECK(ofl_gemm_f32(2, 2, 2, NULL, 2, NULL, 2, NULL, 2, NULL) == OFL_EINVAL);
    CHECK(ofl_gemm_f32(0, 4, 3, NULL, 3, NULL, 4, NULL, 4, NULL) == OFL_OK);
    {
        float dummy[4];
        CHECK(ofl_gemm_f32(1, 1, 1, dummy, 1, dummy, 1, dummy + 2, 1, NULL) == OFL_EDEVICE);
    }

    /* the GA on a synthetic landscape */
    uint32_t target = 0x5au;
    ofl_ga_params ga = {16, 15, 7ull, 0.9, 0.08, 1, 1, 1, 1e-5};
    ofl_ga_result res;
    CHECK(ofl_ga_search(8, &ga, 0u, ga_eval, &target, &res) == OFL_OK);
    CHECK(res.best_gene == target && res.best_time == 1.0 && res.rejected > 0);
    CHECK(ofl_ga_search(31, &ga, 0u, ga_eval, &target, &res) == OFL_EINVAL);
    CHECK(ofl_ga_search(8, &ga, 0u, NULL, &target, &res) == OFL_EINVAL);
    printf("abi_check: all host paths ok\n");
    return 0;
}
