/*
 * Memory and undefined-behaviour check of the CPU oracles (test infrastructure): this driver is
 * compiled together with oracle/vbx_oracle.c and oracle/esdf_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py) and runs every entry point over seeded
 * frames in every mode: simple and grouped raycasting, constant and quadratic weights, binary32
 * and both 16-bit storages, Eq. (1) and the distance along the ray, the band and the whole ray,
 * colour, projection mapping, the traversal and the group mean, and the ESDF oracle with both
 * queues over several incremental updates.  It checks plain invariants (finite values, weights
 * non-negative, |D| within the truncation distance, ESDF distances within d_max) and prints
 * "ALL OK"; any sanitizer report ends the run with an error.
 */
#include "../oracle/vbx_oracle.c"

#include <stdio.h>

/* the ESDF oracle (its own translation unit) */
typedef struct orc_esdf orc_esdf;
orc_esdf* orc_esdf_create(double voxel_size, double gamma, double d_max, int priority);
void orc_esdf_destroy(orc_esdf* E);
void orc_esdf_update(orc_esdf* E, size_t n, const int32_t* coords, const double* d, const double* w);
size_t orc_esdf_export(const orc_esdf* E, int32_t* coords, double* d, uint8_t* info, size_t cap);
void orc_esdf_counts(const orc_esdf* E, uint64_t out[3]);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* splitmix64 -> [0, 1) */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;
#define CHECK(c, ...)                       \
    do {                                    \
        if (!(c)) {                         \
            printf("FAIL: " __VA_ARGS__);   \
            printf("\n");                   \
            ++failures;                     \
        }                                   \
    } while (0)

/* An organised W x H frame in the sensor frame: a wall at depth 2-4 m with bumps, some NaN and
 * some points beyond the range. */
static void make_frame(float* pts, uint32_t* col, int W, int H, int k) {
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            const int idx = i + W * j;
            const double x = (i + 0.5 - W / 2.0) / (W * 0.6), y = (j + 0.5 - H / 2.0) / (W * 0.6);
            double z = 2.0 + 0.3 * sin(0.2 * i + 0.1 * k) + 0.2 * cos(0.3 * j) + 0.01 * urand();
            if (urand() < 0.03) z = 9.0; /* beyond the range */
            pts[3 * idx] = (float)(x * z);
            pts[3 * idx + 1] = (float)(y * z);
            pts[3 * idx + 2] = (float)z;
            if (urand() < 0.05) pts[3 * idx] = NAN;
            col[idx] = (uint32_t)(urand() * 4294967296.0);
        }
}

static void make_pose(float pose[12], int k) {
    const double a = 0.05 * k, c = cos(a), s = sin(a);
    const float R[9] = {(float)c, 0.f, (float)s, 0.f, 1.f, 0.f, (float)-s, 0.f, (float)c};
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) pose[4 * r + q] = R[3 * r + q];
        pose[4 * r + 3] = (float)(0.1 * k * (r == 0) - 0.05 * (r == 1));
    }
}

static void check_export(orc_map* m, const orc_params* P, const char* what) {
    const size_t nb = orc_num_blocks(m);
    int32_t* coords = (int32_t*)malloc((nb + 1) * 3 * sizeof(int32_t));
    double* D = (double*)malloc((nb + 1) * 4096 * sizeof(double));
    double* Wt = (double*)malloc((nb + 1) * 4096 * sizeof(double));
    double* M = (double*)malloc((nb + 1) * 4096 * sizeof(double));
    double* R = (double*)malloc((nb + 1) * 4096 * sizeof(double));
    uint32_t* C = (uint32_t*)malloc((nb + 1) * 4096 * sizeof(uint32_t));
    CHECK(orc_export(m, coords, D, Wt, M, nb) == nb, "%s: export count", what);
    CHECK(orc_export_ramp(m, R, nb) == nb, "%s: ramp export count", what);
    CHECK(orc_export_color(m, C, nb) == nb, "%s: colour export count", what);
    for (size_t i = 0; i < nb * 4096; ++i) {
        CHECK(isfinite(D[i]) && isfinite(Wt[i]) && Wt[i] >= 0.0, "%s: voxel %zu not finite", what, i);
        CHECK(fabs(D[i]) <= (double)P->trunc * (1.0 + 1e-6), "%s: |D| above trunc at %zu", what, i);
        CHECK(M[i] >= 0.0 && R[i] >= 0.0 && R[i] <= M[i] * (1.0 + 1e-12), "%s: diagnostics at %zu", what, i);
        CHECK((C[i] >> 24) == 0, "%s: colour alpha at %zu", what, i);
    }
    int32_t tc[3 * 64];
    uint32_t tn[64];
    (void)orc_last_touches(m, tc, tn, 64);
    orc_stats st;
    orc_last_stats(m, &st);
    free(coords); free(D); free(Wt); free(M); free(R); free(C);
}

static void run_integration(void) {
    const int W = 48, H = 32, N = W * H;
    float* pts = (float*)malloc((size_t)N * 3 * sizeof(float));
    uint32_t* col = (uint32_t*)malloc((size_t)N * sizeof(uint32_t));
    for (int merge = 0; merge < 2; ++merge)
        for (int weighting = 0; weighting < 2; ++weighting)
            for (int fp16 = 0; fp16 < 3; ++fp16)
                for (int dist = 0; dist < 2; ++dist)
                    for (int full = 0; full < 2; ++full)
                        for (int color = 0; color < 2; ++color) {
                            orc_params P;
                            memset(&P, 0, sizeof P);
                            P.voxel_size = 0.1f;
                            P.trunc = 0.3f;
                            P.w_max = weighting ? 50.0f : 3.0f; /* saturates within the frames */
                            P.max_range = 5.0f;
                            P.z_min = 0.1f;
                            P.weighting = weighting;
                            P.merge = merge;
                            P.fp16 = fp16;
                            P.dist = dist;
                            P.full_ray = full;
                            P.color = color;
                            char what[96];
                            snprintf(what, sizeof what, "m%d w%d s%d d%d f%d c%d", merge, weighting, fp16, dist,
                                     full, color);
                            orc_map* m = orc_create(&P);
                            for (int k = 0; k < 3; ++k) {
                                float pose[12];
                                make_frame(pts, col, W, H, k);
                                make_pose(pose, k);
                                orc_stats st;
                                if (color) orc_integrate_color(m, pts, col, (size_t)N, pose, &st);
                                else orc_integrate(m, pts, (size_t)N, pose, &st);
                                CHECK(st.points == (uint64_t)N && st.valid + st.invalid + st.out_of_bounds <= (uint64_t)N,
                                      "%s: statistics", what);
                            }
                            /* an empty frame and a frame of one point */
                            float pose0[12];
                            make_pose(pose0, 0);
                            orc_stats st0;
                            orc_integrate(m, pts, 0, pose0, &st0);
                            orc_integrate(m, pts, 1, pose0, &st0);
                            check_export(m, &P, what);
                            orc_destroy(m);
                        }
    /* projection mapping, organised frames */
    for (int weighting = 0; weighting < 2; ++weighting) {
        orc_params P;
        memset(&P, 0, sizeof P);
        P.voxel_size = 0.1f;
        P.trunc = 0.3f;
        P.w_max = 1e4f;
        P.max_range = 5.0f;
        P.z_min = 0.1f;
        P.weighting = weighting;
        orc_map* m = orc_create(&P);
        const float intr[4] = {W * 0.6f, W * 0.6f, W / 2.0f, H / 2.0f};
        for (int k = 0; k < 3; ++k) {
            float pose[12];
            make_frame(pts, col, W, H, k);
            make_pose(pose, k);
            orc_stats st;
            CHECK(orc_integrate_projective(m, pts, (size_t)N, (uint32_t)W, pose, intr, &st) == 0, "projective");
        }
        orc_stats st;
        float pose[12];
        make_pose(pose, 0);
        CHECK(orc_integrate_projective(m, pts, (size_t)N, 7u, pose, intr, &st) != 0, "projective ragged width");
        check_export(m, &P, "projective");
        orc_destroy(m);
    }
    free(pts);
    free(col);
}

static void run_traversal_and_means(void) {
    int32_t buf[3 * 400];
    for (int t = 0; t < 2000; ++t) {
        float A[3], B[3];
        for (int k = 0; k < 3; ++k) {
            A[k] = (float)((urand() - 0.5) * 40.0);
            B[k] = A[k] + (float)((urand() - 0.5) * 60.0);
        }
        const int n = orc_dda(A, B, buf, 400);
        CHECK(n >= 1, "dda count");
        (void)orc_dda(A, B, buf, 3); /* a buffer shorter than the walk */
    }
    float p[3 * 64], w[64], out[3];
    for (int i = 0; i < 64; ++i) {
        for (int k = 0; k < 3; ++k) p[3 * i + k] = (float)(1.23 + 0.05 * urand());
        w[i] = (float)(0.01 + urand());
    }
    orc_group_mean(p, w, 64, 0.1f, 25, out);
    orc_group_mean(p, w, 1, 0.1f, 0, out);
    for (int k = 0; k < 3; ++k) CHECK(isfinite(out[k]), "group mean");
    for (int i = 0; i < 1000; ++i) CHECK(isfinite(orc_round_half((urand() - 0.5) * 2e5)), "round half");
}

static void run_esdf(void) {
    const int S = 20, NV = S * S * S;
    int32_t* c = (int32_t*)malloc((size_t)NV * 3 * sizeof(int32_t));
    double* d = (double*)malloc((size_t)NV * sizeof(double));
    double* w = (double*)malloc((size_t)NV * sizeof(double));
    for (int q = 0; q < 2; ++q) {
        orc_esdf* E = orc_esdf_create(0.1, 0.1, 1.5, q);
        for (int round = 0; round < 4; ++round) {
            int n = 0;
            for (int z = 0; z < S; ++z)
                for (int y = 0; y < S; ++y)
                    for (int x = 0; x < S; ++x) {
                        if (round > 0 && urand() < 0.7) continue; /* later rounds change a part */
                        c[3 * n] = x - S / 2;
                        c[3 * n + 1] = y - S / 2;
                        c[3 * n + 2] = z - 3;
                        const double plane = (z - 3 + 0.5) * 0.1 - 0.25 - 0.05 * round;
                        d[n] = plane < -0.3 ? -0.3 : (plane > 0.3 ? 0.3 : plane);
                        w[n] = urand() < 0.1 ? 0.0 : 1.0;
                        ++n;
                    }
            orc_esdf_update(E, (size_t)n, c, d, w);
        }
        const size_t ne = orc_esdf_export(E, NULL, NULL, NULL, 0);
        int32_t* ec = (int32_t*)malloc((ne + 1) * 3 * sizeof(int32_t));
        double* ed = (double*)malloc((ne + 1) * sizeof(double));
        uint8_t* ei = (uint8_t*)malloc(ne + 1);
        CHECK(orc_esdf_export(E, ec, ed, ei, ne) == ne, "esdf export count");
        for (size_t i = 0; i < ne; ++i) CHECK(isfinite(ed[i]) && fabs(ed[i]) <= 1.5 + 1e-9, "esdf distance");
        uint64_t counts[3];
        orc_esdf_counts(E, counts);
        free(ec); free(ed); free(ei);
        orc_esdf_destroy(E);
    }
    free(c); free(d); free(w);
}

int main(void) {
    run_integration();
    run_traversal_and_means();
    run_esdf();
    if (failures) {
        printf("%d failures\n", failures);
        return 1;
    }
    printf("ALL OK\n");
    return 0;
}
