/*
 * Drives every entry point of the CPU oracle on small instances, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (the oracle source is
 * included whole, so its internal functions build with the same flags).  Each
 * call must succeed and leave consistent results: energies equal to the
 * recomputed energy of their states, E(s) = E'(s') + offset for reductions and
 * completions.  Exit status 0 when every check holds; a sanitizer report
 * aborts with a nonzero status.
 */
#include "../../oracle/spvar_oracle.c"

#include <stdio.h>

static int failures = 0;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);       \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

/* A problem with owned arrays. */
typedef struct {
    orc_problem p;
    int32_t *rp, *col, *J, *h;
    uint8_t *colour;
} owned;

static uint64_t lcg(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return *s >> 33;
}

/* Symmetric CSR from an undirected edge list (i < j), coloured by Jones-Plassmann. */
static owned make_graph(int32_t n, int32_t m, const int32_t *ei, const int32_t *ej, const int32_t *w,
                        const int32_t *h, int32_t scale)
{
    owned g;
    int32_t *deg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t)), i, k;
    memset(&g, 0, sizeof g);
    for (k = 0; k < m; ++k) {
        ++deg[ei[k]];
        ++deg[ej[k]];
    }
    g.rp = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    g.rp[0] = 0;
    for (i = 0; i < n; ++i)
        g.rp[i + 1] = g.rp[i] + deg[i];
    g.col = (int32_t *)malloc(sizeof(int32_t) * ((size_t)2 * m + 1));
    g.J = (int32_t *)malloc(sizeof(int32_t) * ((size_t)2 * m + 1));
    g.h = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    g.colour = (uint8_t *)malloc((size_t)n + 1);
    /* fill rows in increasing column order: insertion sort per row */
    for (i = 0; i < n; ++i)
        deg[i] = 0;
    for (k = 0; k < m; ++k) {
        int32_t a = ei[k], b = ej[k], pa = g.rp[a] + deg[a]++, pb = g.rp[b] + deg[b]++;
        g.col[pa] = b;
        g.J[pa] = w[k];
        g.col[pb] = a;
        g.J[pb] = w[k];
    }
    for (i = 0; i < n; ++i) {
        int32_t x, y;
        for (x = g.rp[i] + 1; x < g.rp[i + 1]; ++x)
            for (y = x; y > g.rp[i] && g.col[y - 1] > g.col[y]; --y) {
                int32_t tc = g.col[y], tj = g.J[y];
                g.col[y] = g.col[y - 1];
                g.J[y] = g.J[y - 1];
                g.col[y - 1] = tc;
                g.J[y - 1] = tj;
            }
        g.h[i] = h[i];
    }
    free(deg);
    g.p.n = n;
    g.p.row_ptr = g.rp;
    g.p.col = g.col;
    g.p.J = g.J;
    g.p.h = g.h;
    g.p.colour = g.colour;
    g.p.n_colours = 1;
    g.p.scale_log2 = scale;
    {
        int32_t nc = 0;
        int rc = orc_colour_jp(&g.p, 7, g.colour, &nc, 16);
        CHECK(rc == ORC_OK);
        g.p.n_colours = nc;
    }
    return g;
}

static void free_graph(owned *g)
{
    free(g->rp);
    free(g->col);
    free(g->J);
    free(g->h);
    free(g->colour);
}

/* Periodic cubic L^3 lattice with random couplers in [-jmax, jmax] \ {0}, biases in [-hmax, hmax]. */
static owned cubic(int32_t L, int32_t jmax, int32_t hmax, int32_t scale, uint64_t seed)
{
    int32_t n = L * L * L, m = 3 * n, x, y, z, k = 0;
    int32_t *ei = (int32_t *)malloc(sizeof(int32_t) * m), *ej = (int32_t *)malloc(sizeof(int32_t) * m);
    int32_t *w = (int32_t *)malloc(sizeof(int32_t) * m), *h = (int32_t *)malloc(sizeof(int32_t) * n);
    owned g;
    for (z = 0; z < L; ++z)
        for (y = 0; y < L; ++y)
            for (x = 0; x < L; ++x) {
                int32_t i = x + L * (y + L * z), nb[3], d;
                nb[0] = (x + 1) % L + L * (y + L * z);
                nb[1] = x + L * ((y + 1) % L + L * z);
                nb[2] = x + L * (y + L * ((z + 1) % L));
                for (d = 0; d < 3; ++d) {
                    int32_t v = (int32_t)(lcg(&seed) % (uint64_t)(2 * jmax)) - jmax;
                    ei[k] = i < nb[d] ? i : nb[d];
                    ej[k] = i < nb[d] ? nb[d] : i;
                    w[k] = v >= 0 ? v + 1 : v;
                    ++k;
                }
                h[i] = hmax ? (int32_t)(lcg(&seed) % (uint64_t)(2 * hmax + 1)) - hmax : 0;
            }
    g = make_graph(n, m, ei, ej, w, h, scale);
    free(ei);
    free(ej);
    free(w);
    free(h);
    return g;
}

/* A random tree hanging off a 4-cycle (the tree step removes the tree). */
static owned tree_on_cycle(int32_t n, uint64_t seed)
{
    int32_t m = n, k, v;
    int32_t *ei = (int32_t *)malloc(sizeof(int32_t) * m), *ej = (int32_t *)malloc(sizeof(int32_t) * m);
    int32_t *w = (int32_t *)malloc(sizeof(int32_t) * m), *h = (int32_t *)malloc(sizeof(int32_t) * n);
    owned g;
    for (k = 0; k < 4; ++k) {
        ei[k] = k < 3 ? k : 0;
        ej[k] = k < 3 ? k + 1 : 3;
    }
    for (v = 4; v < n; ++v) {
        ei[v] = (int32_t)(lcg(&seed) % (uint64_t)v);
        ej[v] = v;
    }
    for (k = 0; k < m; ++k) {
        int32_t x = (int32_t)(lcg(&seed) % 6) - 3;
        w[k] = x >= 0 ? x + 1 : x;
    }
    for (v = 0; v < n; ++v)
        h[v] = (int32_t)(lcg(&seed) % 5) - 2;
    g = make_graph(n, m, ei, ej, w, h, 0);
    free(ei);
    free(ej);
    free(w);
    free(h);
    return g;
}

static void linear_betas(double *b, int32_t s, double b0, double b1)
{
    int32_t t;
    for (t = 0; t < s; ++t)
        b[t] = s > 1 ? b0 + (b1 - b0) * t / (s - 1) : b1;
}

static void check_energies(const orc_problem *P, const int8_t *S, const int64_t *E, int32_t R)
{
    int32_t r;
    for (r = 0; r < R; ++r)
        CHECK(E[r] == orc_energy(P, S + (size_t)r * P->n));
}

static void test_sa_persist_tree(void)
{
    owned g = cubic(4, 2, 2, 0, 11);
    const int32_t n = g.p.n, R = 40, S = 60;
    double betas[60];
    int8_t *sp = (int8_t *)malloc((size_t)R * n), *full = (int8_t *)malloc((size_t)R * n);
    int64_t E[40], info[8];
    uint8_t fm[64], kind[64];
    int8_t fv[64], val[64];
    int32_t rp[65], col[384], J[384], h[64], orig[64], parent[64], round[64], comp[64];
    uint8_t co[64];
    orc_problem red;
    int32_t r, i, nc;
    linear_betas(betas, S, 0.1, 3.0);
    CHECK(orc_sa_sample(&g.p, betas, S, 5, 0, 0, R, NULL, NULL, sp, E) == ORC_OK);
    check_energies(&g.p, sp, E, R);
    for (i = 0; i <= 2; ++i) {
        CHECK(orc_persist_fix(&g.p, sp, E, R, 0.25, 1.0, i, fm, fv, rp, col, J, h, co, orig, info) == ORC_OK);
        red = g.p;
        red.n = (int32_t)info[0];
        red.row_ptr = rp;
        red.col = col;
        red.J = J;
        red.h = h;
        red.colour = co;
        /* E(s) = E'(s_U) + offset for every sample row that agrees with the fixes */
        for (r = 0; r < R; ++r) {
            int8_t sub[64], ok = 1;
            int32_t u;
            for (u = 0; u < n; ++u)
                if (fm[u] && sp[(size_t)r * n + u] != fv[u])
                    ok = 0;
            if (!ok)
                continue;
            for (u = 0; u < red.n; ++u)
                sub[u] = sp[(size_t)r * n + orig[u]];
            CHECK(orc_energy(&g.p, sp + (size_t)r * n) == orc_energy(&red, sub) + info[2]);
        }
    }
    nc = orc_components(&g.p, comp);
    CHECK(nc >= 1);
    {
        int8_t *mg = (int8_t *)malloc((size_t)R * n);
        int64_t mE[40], pe[64 * 40];
        CHECK(orc_merge_sorted(&g.p, comp, nc, sp, R, mg, mE, pe) == ORC_OK);
        check_energies(&g.p, mg, mE, R);
        free(mg);
    }
    free_graph(&g);

    g = tree_on_cycle(40, 3);
    CHECK(orc_tree_peel(&g.p, kind, val, parent, round, rp, col, J, h, co, orig, info) == ORC_OK);
    red = g.p;
    red.n = (int32_t)info[0];
    red.row_ptr = rp;
    red.col = col;
    red.J = J;
    red.h = h;
    red.colour = co;
    {
        int8_t reduced[8 * 4];
        int32_t u;
        for (r = 0; r < 8; ++r)
            for (u = 0; u < red.n; ++u)
                reduced[r * red.n + u] = (int8_t)((r >> (u % 3)) & 1 ? 1 : -1);
        CHECK(orc_tree_expand(g.p.n, kind, val, parent, round, orig, red.n, (int32_t)info[5], reduced, 8, full) ==
              ORC_OK);
        for (r = 0; r < 8; ++r)
            CHECK(orc_energy(&g.p, full + (size_t)r * g.p.n) == orc_energy(&red, reduced + r * red.n) + info[2]);
    }
    free_graph(&g);
    free(sp);
    free(full);
}

static void test_ispvar_and_multistart(void)
{
    owned g = cubic(4, 1, 0, 0, 21);
    const int32_t n = g.p.n;
    double betas[50];
    uint8_t fm[64];
    int8_t fv[64];
    int64_t rinfo[3 * 4];
    int32_t run;
    linear_betas(betas, 50, 0.1, 3.0);
    run = orc_ispvar(&g.p, betas, 50, 30, 9, 3, 0.2, 1.0, 2, fm, fv, rinfo);
    CHECK(run >= 1);
    {
        enum { S = 3, RC = 20, F = 15, RS = 15 };
        orc_ms_params p;
        orc_ms_out o;
        int64_t cE[S * RC], fE[S * F], sE[S * RS], info[S * 8], pre[8], sb[S], best = 0;
        uint8_t mfm[S * 64];
        int8_t mfv[S * 64], bs[64];
        int32_t order;
        for (order = 0; order < 2; ++order) {
            memset(&p, 0, sizeof p);
            p.betas = betas;
            p.sweeps = 50;
            p.seed = 13;
            p.starts = S;
            p.corr_reads = RC;
            p.fixing_reads = F;
            p.solving_reads = RS;
            p.elite_frac = 0.2;
            p.threshold = 1.0;
            p.gauge = 0;
            p.corr_elite_frac = 0.3;
            p.corr_threshold = 1.0;
            p.corr_after = order;
            p.preprocess = 3;
            p.merge = 1;
            o.corr_E = cE;
            o.fixing_E = fE;
            o.solving_E = sE;
            o.fixed_mask = mfm;
            o.fixed_val = mfv;
            o.info = info;
            o.info_pre = pre;
            o.start_best = sb;
            o.best_spins = bs;
            o.best_E = &best;
            CHECK(orc_multistart(&g.p, &p, &o) == ORC_OK);
            CHECK(best == orc_energy(&g.p, bs));
        }
    }
    {
        int64_t sb[4] = {-3, -5, -5, -4};
        double pr = 0.0;
        CHECK(orc_r99(sb, 4, -5, 100.0, &pr) > 0.0 && pr == 0.5);
    }
    (void)n;
    free_graph(&g);
}

static void test_pt_sqa(void)
{
    owned g = cubic(4, 1000, 0, 10, 31); /* two-digit tables at scale 2^10 */
    const int32_t n = g.p.n, K = 6, runs = 2, chains = 2, sweeps = 40, half = K / 2;
    double betas[6];
    int8_t *fs = (int8_t *)malloc((size_t)runs * chains * K * n);
    int8_t *ts = (int8_t *)malloc((size_t)runs * chains * half * TOPK * n);
    int64_t fE[2 * 2 * 6], tE[2 * 2 * 3 * TOPK];
    int32_t tc[2 * 2 * 3], k, tt;
    for (k = 0; k < K; ++k)
        betas[k] = 0.2 * pow(25.0, (double)k / (K - 1));
    for (tt = 1; tt <= 2; ++tt) {
        orc_set_slot_threads(tt);
        CHECK(orc_pt_sample(&g.p, betas, K, runs, chains, sweeps, 3, 0, 0, K, 0, runs, fs, fE, ts, tE, tc, NULL,
                            NULL, NULL, NULL, NULL, NULL) == ORC_OK);
        check_energies(&g.p, fs, fE, runs * chains * K);
    }
    orc_set_slot_threads(1);
    {
        /* a run stopped after 15 sweeps and resumed from its checkpoint equals the 40-sweep run */
        int8_t *fs2 = (int8_t *)malloc((size_t)runs * chains * K * n);
        int8_t *ts2 = (int8_t *)malloc((size_t)runs * chains * half * TOPK * n);
        int64_t fE2[2 * 2 * 6], tE2[2 * 2 * 3 * TOPK];
        int32_t tc2[2 * 2 * 3];
        CHECK(orc_pt_sample(&g.p, betas, K, runs, chains, 15, 3, 0, 0, K, 0, runs, fs2, fE2, ts2, tE2, tc2, NULL,
                            NULL, NULL, NULL, NULL, NULL) == ORC_OK);
        CHECK(orc_pt_sample(&g.p, betas, K, runs, chains, sweeps - 15, 3, 15, 0, K, 0, runs, fs2, fE2, ts2, tE2,
                            tc2, NULL, NULL, fs2, ts2, tE2, tc2) == ORC_OK);
        CHECK(memcmp(fs, fs2, (size_t)runs * chains * K * n) == 0 && memcmp(fE, fE2, sizeof fE) == 0);
        CHECK(memcmp(ts, ts2, (size_t)runs * chains * half * TOPK * n) == 0 && memcmp(tE, tE2, sizeof tE) == 0 &&
              memcmp(tc, tc2, sizeof tc) == 0);
        free(fs2);
        free(ts2);
    }
    {
        const int32_t P = 8, R = 6, sw = 20;
        double b[20], gm[20];
        int8_t *spins = (int8_t *)malloc((size_t)R * n);
        int64_t E[6];
        int32_t bestk[6], t;
        for (t = 0; t < sw; ++t) {
            b[t] = 0.2 + 2.8 * t / (sw - 1);
            gm[t] = 3.0 * pow(0.02, (double)t / (sw - 1));
        }
        CHECK(orc_sqa_sample(&g.p, b, gm, sw, P, 5, 0, R, NULL, NULL, spins, E, bestk) == ORC_OK);
        check_energies(&g.p, spins, E, R);
        free(spins);
    }
    free(fs);
    free(ts);
    free_graph(&g);
}

int main(void)
{
    test_sa_persist_tree();
    test_ispvar_and_multistart();
    test_pt_sqa();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: all checks passed\n");
    return 0;
}
