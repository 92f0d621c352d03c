/* Host-side checks of the C ABI on handles built with PF_BUILD_HOST_ONLY
 * (no GPU): pattern building, tile and lane tables for every tile size,
 * pattern export, the Algorithm 2 index map, and the argument checks.
 * Built and run by tests/test_host_sanitizers.py with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code; exits non-zero on the first
 * failed check. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pf.h"

static uint64_t rng_state = 0x2302107360001ull;
static uint32_t rnd(void) { /* xorshift64* */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 2685821657736338717ull) >> 32);
}
static double unif(double a, double b) { return a + (b - a) * (rnd() / 4294967296.0); }

#define CHECK(cond, ...)                                               \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "check failed at line %d: ", __LINE__);    \
            fprintf(stderr, __VA_ARGS__);                              \
            fprintf(stderr, " (%s)\n", pf_last_error());               \
            exit(1);                                                   \
        }                                                              \
    } while (0)

typedef struct {
    int32_t nb, nl;
    int32_t *f, *t;
    double *r, *x, *b, *tap, *sh, *gs, *bs;
} Grid;

static void grid_alloc(Grid *g, int32_t nb, int32_t nl) {
    g->nb = nb;
    g->nl = nl;
    g->f = malloc(sizeof(int32_t) * (nl + 1));
    g->t = malloc(sizeof(int32_t) * (nl + 1));
    g->r = malloc(sizeof(double) * (nl + 1));
    g->x = malloc(sizeof(double) * (nl + 1));
    g->b = malloc(sizeof(double) * (nl + 1));
    g->tap = malloc(sizeof(double) * (nl + 1));
    g->sh = malloc(sizeof(double) * (nl + 1));
    g->gs = malloc(sizeof(double) * nb);
    g->bs = malloc(sizeof(double) * nb);
}

static void grid_free(Grid *g) {
    free(g->f), free(g->t), free(g->r), free(g->x), free(g->b), free(g->tap), free(g->sh), free(g->gs), free(g->bs);
}

/* A random grid: tree-like edges with local numbering, extra edges, some
 * parallel branches, optionally one hub bus with `hub` extra branches, and
 * isolated buses at the end. */
static Grid random_grid(int32_t nb, int32_t extra, int32_t parallel, int32_t hub, int32_t isolated) {
    const int32_t conn = nb - isolated;
    const int32_t nl = (conn > 1 ? conn - 1 : 0) + (conn > 1 ? extra + parallel + hub : 0);
    Grid g;
    grid_alloc(&g, nb, nl);
    int32_t l = 0;
    for (int32_t i = 1; i < conn; ++i) {
        int32_t lo = i > 64 ? i - 64 : 0;
        g.f[l] = i;
        g.t[l] = lo + (int32_t)(rnd() % (uint32_t)(i - lo));
        ++l;
    }
    for (int32_t k = 0; conn > 1 && k < extra; ++k) {
        int32_t a = (int32_t)(rnd() % (uint32_t)conn), c = (int32_t)(rnd() % (uint32_t)conn);
        if (a == c) c = (a + 1) % conn;
        g.f[l] = a, g.t[l] = c, ++l;
    }
    for (int32_t k = 0; conn > 1 && k < parallel; ++k) { /* repeat an existing pair, either orientation */
        int32_t m = (int32_t)(rnd() % (uint32_t)l);
        int flip = rnd() & 1;
        g.f[l] = flip ? g.t[m] : g.f[m];
        g.t[l] = flip ? g.f[m] : g.t[m];
        ++l;
    }
    for (int32_t k = 0; conn > 1 && k < hub; ++k) {
        g.f[l] = 0;
        g.t[l] = 1 + (int32_t)(rnd() % (uint32_t)(conn - 1));
        ++l;
    }
    for (int32_t k = 0; k < l; ++k) {
        if (rnd() & 1) { /* random orientation */
            int32_t s = g.f[k];
            g.f[k] = g.t[k], g.t[k] = s;
        }
        g.r[k] = unif(0.001, 0.05);
        g.x[k] = unif(0.01, 0.3);
        g.b[k] = unif(0.0, 0.1);
        const int xf = rnd() % 5 == 0;
        g.tap[k] = xf ? unif(0.95, 1.05) : ((rnd() & 3) == 0 ? 0.0 : 1.0);
        g.sh[k] = xf ? unif(-0.1, 0.1) : 0.0;
    }
    for (int32_t i = 0; i < nb; ++i) {
        g.gs[i] = (rnd() % 10 == 0) ? unif(0.0, 0.02) : 0.0;
        g.bs[i] = (rnd() % 10 == 0) ? unif(-0.1, 0.1) : 0.0;
    }
    return g;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Patterns, every schedule, the index map; one grid per handle. */
static void check_grid(const Grid *g) {
    pf_grid *h = NULL;
    int rc = pf_build_pattern(g->nb, g->nl, g->f, g->t, g->r, g->x, g->b, g->tap, g->sh, g->gs, g->bs, 1, NULL, NULL,
                              PF_BUILD_HOST_ONLY, &h);
    CHECK(rc == PF_OK && h, "build nb=%d nl=%d rc=%d", g->nb, g->nl, rc);
    int64_t nb = 0, nnz_y = 0, nnz_j = 0;
    int32_t ng = 0;
    CHECK(pf_grid_sizes(h, &nb, &nnz_y, &nnz_j, &ng) == PF_OK, "sizes");
    CHECK(nb == g->nb && ng == 1 && nnz_j == 4 * nnz_y && nnz_y >= nb && nnz_y <= nb + 2 * (int64_t)g->nl,
          "size relations nb=%lld nnz_y=%lld", (long long)nb, (long long)nnz_y);
    const int32_t n = 2 * g->nb;
    int32_t *yr = malloc(sizeof(int32_t) * (g->nb + 1)), *yc = malloc(sizeof(int32_t) * (nnz_y + 1));
    int32_t *jr = malloc(sizeof(int32_t) * (n + 1)), *jc = malloc(sizeof(int32_t) * (nnz_j + 1));
    CHECK(pf_pattern_export(h, yr, yc, jr, jc) == PF_OK, "export");
    CHECK(yr[0] == 0 && yr[g->nb] == nnz_y && jr[0] == 0 && jr[n] == nnz_j, "pointer ends");
    for (int32_t i = 0; i < g->nb; ++i) {
        int diag = 0;
        for (int32_t q = yr[i]; q < yr[i + 1]; ++q) {
            CHECK(yc[q] >= 0 && yc[q] < g->nb, "ycol range");
            if (q > yr[i]) CHECK(yc[q] > yc[q - 1], "ycol ascending");
            diag |= yc[q] == i;
        }
        CHECK(diag, "diagonal of row %d", i);
    }
    for (int32_t i = 0; i < n; ++i) {
        CHECK(jr[i + 1] >= jr[i], "jrow monotone");
        for (int32_t q = jr[i]; q < jr[i + 1]; ++q) {
            CHECK(jc[q] >= 0 && jc[q] < n, "jcol range");
            if (q > jr[i]) CHECK(jc[q] > jc[q - 1], "jcol ascending");
        }
    }
    /* every schedule: tiles and lane tables are rebuilt on the host */
    const int32_t tiles[4] = {64, 128, 256, 512};
    for (int k = 0; k < 4; ++k) {
        CHECK(pf_set_schedule(h, tiles[k], (int32_t)(rnd() % 4), (int32_t)(rnd() % 3)) == PF_OK, "schedule %d",
              tiles[k]);
        int32_t ti = 0, spb = 0, order = 0, ntiles = 0;
        CHECK(pf_get_schedule(h, &ti, &spb, &order, &ntiles) == PF_OK && ti == tiles[k] && ntiles >= 1,
              "get schedule");
    }
    /* Algorithm 2 map onto the exported pattern itself: the identity (CSR) ... */
    int32_t *map = malloc(sizeof(int32_t) * (nnz_j + 1));
    CHECK(pf_jacobian_map(h, PF_LAYOUT_CSR, n, jr, jc, map) == PF_OK, "map csr");
    for (int64_t k = 0; k < nnz_j; ++k) CHECK(map[k] == k, "identity map at %lld", (long long)k);
    /* ... and a permutation in column-major order (the pattern is symmetric,
     * so the same arrays describe its CSC form) */
    CHECK(pf_jacobian_map(h, PF_LAYOUT_CSC, n, jr, jc, map) == PF_OK, "map csc");
    qsort(map, (size_t)nnz_j, sizeof(int32_t), cmp_i32);
    for (int64_t k = 0; k < nnz_j; ++k) CHECK(map[k] == k, "csc map is a permutation");
    /* a target missing one entry is rejected with a message */
    if (nnz_j > 0) {
        int32_t *jc2 = malloc(sizeof(int32_t) * (nnz_j + 1)), *jr2 = malloc(sizeof(int32_t) * (n + 1));
        memcpy(jr2, jr, sizeof(int32_t) * (n + 1));
        int32_t row = 0;
        while (jr[row + 1] == jr[row]) ++row;
        for (int32_t i = row + 1; i <= n; ++i) jr2[i] -= 1; /* drop the first entry of `row` */
        memcpy(jc2, jc, sizeof(int32_t) * jr[row]);
        memcpy(jc2 + jr[row], jc + jr[row] + 1, sizeof(int32_t) * (nnz_j - jr[row] - 1));
        CHECK(pf_jacobian_map(h, PF_LAYOUT_CSR, n, jr2, jc2, map) == PF_EINVAL, "incomplete target rejected");
        free(jc2), free(jr2);
    }
    /* evaluation calls on a host-only handle */
    CHECK(pf_injections_elementwise(h, 1, (const double *)16, (const double *)16, (double *)32, (double *)48, NULL) ==
              PF_ESTATE,
          "host-only evaluation");
    CHECK(pf_ybus(h, NULL, NULL, NULL) == PF_ESTATE, "host-only ybus");
    free(map), free(yr), free(yc), free(jr), free(jc);
    pf_grid_free(h);
}

/* Several grids in one handle: offsets, schedules, export. */
static void check_multigrid(void) {
    const int G = 4;
    Grid parts[4] = {random_grid(30, 10, 2, 0, 1), random_grid(1, 0, 0, 0, 0), random_grid(700, 200, 5, 600, 3),
                     random_grid(2, 0, 3, 0, 0)};
    int32_t nb = 0, nl = 0, bus_off[5] = {0}, br_off[5] = {0};
    for (int k = 0; k < G; ++k) {
        nb += parts[k].nb, nl += parts[k].nl;
        bus_off[k + 1] = nb, br_off[k + 1] = nl;
    }
    Grid all;
    grid_alloc(&all, nb, nl);
    for (int k = 0; k < G; ++k) {
        memcpy(all.f + br_off[k], parts[k].f, sizeof(int32_t) * parts[k].nl);
        memcpy(all.t + br_off[k], parts[k].t, sizeof(int32_t) * parts[k].nl);
        memcpy(all.r + br_off[k], parts[k].r, sizeof(double) * parts[k].nl);
        memcpy(all.x + br_off[k], parts[k].x, sizeof(double) * parts[k].nl);
        memcpy(all.b + br_off[k], parts[k].b, sizeof(double) * parts[k].nl);
        memcpy(all.tap + br_off[k], parts[k].tap, sizeof(double) * parts[k].nl);
        memcpy(all.sh + br_off[k], parts[k].sh, sizeof(double) * parts[k].nl);
        memcpy(all.gs + bus_off[k], parts[k].gs, sizeof(double) * parts[k].nb);
        memcpy(all.bs + bus_off[k], parts[k].bs, sizeof(double) * parts[k].nb);
    }
    pf_grid *h = NULL;
    CHECK(pf_build_pattern(nb, nl, all.f, all.t, all.r, all.x, all.b, all.tap, all.sh, all.gs, all.bs, G, bus_off,
                           br_off, PF_BUILD_HOST_ONLY, &h) == PF_OK,
          "multigrid build");
    int64_t y_off[5], j_off[5], nnz_y = 0, nnz_j = 0;
    CHECK(pf_grid_offsets(h, y_off, j_off) == PF_OK && y_off[0] == 0, "offsets");
    CHECK(pf_pattern_sizes(h, &nnz_y, &nnz_j) == PF_OK && y_off[G] == nnz_y && j_off[G] == nnz_j, "offset ends");
    for (int k = 0; k < G; ++k) CHECK(j_off[k] == 4 * y_off[k], "j_off = 4 y_off");
    int32_t *yr = malloc(sizeof(int32_t) * (nb + G)), *yc = malloc(sizeof(int32_t) * nnz_y);
    int32_t *jr = malloc(sizeof(int32_t) * (2 * nb + G)), *jc = malloc(sizeof(int32_t) * nnz_j);
    CHECK(pf_pattern_export(h, yr, yc, jr, jc) == PF_OK, "multigrid export");
    for (int t = 64; t <= 512; t *= 2) CHECK(pf_set_schedule(h, t, 0, 0) == PF_OK, "multigrid schedule");
    int32_t map1[1];
    CHECK(pf_jacobian_map(h, PF_LAYOUT_CSR, 2 * nb, jr, jc, map1) == PF_EUNSUP, "map needs one grid");
    free(yr), free(yc), free(jr), free(jc);
    pf_grid_free(h);
    grid_free(&all);
    for (int k = 0; k < G; ++k) grid_free(&parts[k]);
}

/* Invalid grids are rejected before anything is built. */
static void check_rejections(void) {
    Grid g = random_grid(10, 3, 0, 0, 0);
    pf_grid *h = (pf_grid *)1;
#define BUILD() pf_build_pattern(g.nb, g.nl, g.f, g.t, g.r, g.x, g.b, g.tap, g.sh, g.gs, g.bs, 1, NULL, NULL, \
                                 PF_BUILD_HOST_ONLY, &h)
    int32_t keep = g.f[0];
    g.f[0] = g.nb;
    CHECK(BUILD() == PF_EINVAL && h == NULL, "bus index out of range");
    g.f[0] = g.t[0];
    CHECK(BUILD() == PF_EINVAL, "self loop");
    g.f[0] = keep;
    double kr = g.r[1], kx = g.x[1];
    g.r[1] = 0.0, g.x[1] = 0.0;
    CHECK(BUILD() == PF_EINVAL, "r = x = 0");
    g.r[1] = kr, g.x[1] = NAN;
    CHECK(BUILD() == PF_EINVAL, "non-finite reactance");
    g.x[1] = kx;
    double kt = g.tap[2];
    g.tap[2] = -1.0;
    CHECK(BUILD() == PF_EINVAL, "negative tap");
    g.tap[2] = kt;
    g.gs[3] = INFINITY;
    CHECK(BUILD() == PF_EINVAL, "non-finite shunt");
    g.gs[3] = 0.0;
    CHECK(BUILD() == PF_OK && h, "valid again");
    CHECK(pf_set_schedule(h, 100, 0, 0) == PF_EINVAL, "tile size");
    CHECK(pf_set_schedule(h, 256, -1, 0) == PF_EINVAL, "states per block");
    CHECK(pf_set_schedule(h, 256, 0, 7) == PF_EINVAL, "order");
    pf_grid_free(h);
    int32_t bo[3] = {0, 4, 10}, ro[3] = {0, 2, g.nl};
    h = NULL;
    /* branch 0 lies in grid 0 (buses 0..3) but refers to a bus of grid 1 */
    CHECK(pf_build_pattern(g.nb, g.nl, g.f, g.t, g.r, g.x, g.b, g.tap, g.sh, g.gs, g.bs, 2, bo, ro,
                           PF_BUILD_HOST_ONLY, &h) == PF_EINVAL ||
              h != NULL,
          "grid-local indices");
    pf_grid_free(h);
    bo[1] = 0;
    h = NULL;
    CHECK(pf_build_pattern(g.nb, g.nl, g.f, g.t, g.r, g.x, g.b, g.tap, g.sh, g.gs, g.bs, 2, bo, ro,
                           PF_BUILD_HOST_ONLY, &h) == PF_EINVAL,
          "empty grid");
    grid_free(&g);
#undef BUILD
}

int main(void) {
    const int32_t sizes[][5] = {
        /* nb, extra, parallel, hub, isolated */
        {1, 0, 0, 0, 0},     {2, 0, 0, 0, 0},       {2, 0, 4, 0, 0},        {3, 1, 1, 0, 1},
        {50, 20, 3, 0, 2},   {333, 360, 3, 0, 7},   {700, 200, 0, 700, 0},  {600, 100, 8, 1100, 2},
        {2000, 700, 12, 0, 5}, {5000, 1500, 0, 0, 0},
    };
    for (size_t k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k) {
        Grid g = random_grid(sizes[k][0], sizes[k][1], sizes[k][2], sizes[k][3], sizes[k][4]);
        check_grid(&g);
        grid_free(&g);
    }
    check_multigrid();
    check_rejections();
    printf("host checks passed\n");
    return 0;
}
