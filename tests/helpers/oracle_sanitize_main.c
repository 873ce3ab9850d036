/*
 * Driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * FP64 oracle (test infrastructure): calls every exported oracle routine on
 * small inputs -- the hand-worked example of the section 2.2 terms, random
 * tiny portfolios with and without secondary uncertainty (independent,
 * correlated and sigma-capped rows, both keyings, the occurrence view), the
 * special functions at ordinary and near-Bernoulli shapes, PML / TVaR -- and
 * checks a few facts that hold for any correct run.  Exit status 0 = every
 * check held; the sanitizers abort on the first memory error or undefined
 * behaviour they see.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_ara_run(int64_t n_trials, int64_t trial_base, const int64_t *offsets,
                const int32_t *event_ids, int32_t n_catalogue, int32_t n_layers,
                const double *layer_terms, int32_t n_elt, const int32_t *elt_layer,
                const uint32_t *elt_id, const int64_t *elt_row_off, const double *elt_terms,
                const int32_t *row_event, const float *row_mean, const float *row_sigma_i,
                const float *row_sigma_c, const float *row_max, uint64_t seed,
                int32_t su_enabled, int32_t keying, const uint32_t *layer_program,
                int32_t n_threads, double *ylt, double *ylt_pf, double *gross, int64_t *hits,
                uint64_t *hit_chk, double *occ_view);
int orc_pml_tvar(const double *ylt, int64_t n, const double *rps, int32_t n_rp, double *pml,
                 double *tvar);
double orc_betaincinv_pair(double a, double b, double z, double zc, double *xc);
double orc_betainc(double a, double b, double x);
double orc_norm_quantile(double p);
double orc_norm_cdf(double x);
void orc_beta_fit(double mu, double sigma, double max_l, double *alpha, double *beta);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static uint64_t rng_state = 88172645463325252ull;
static uint32_t rnd(uint32_t n)  /* xorshift64, uniform enough for test shapes */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state % n);
}

static void worked_example(void)
{
    /* events A = 0, B = 1; ELT1 {A: 3e6, B: 5e5}, ELT2 {A: 1e6}; trial [A, B, A] */
    const int64_t off[2] = {0, 3};
    const int32_t ev[3] = {0, 1, 0};
    const double lt[4] = {1e6, 2e7, 5e6, 1e8};
    const int32_t el[2] = {0, 0};
    const uint32_t eid[2] = {0, 1};
    const int64_t ro[3] = {0, 2, 3};
    const double et[6] = {1e5, 5e6, 1.0, 1e5, 5e6, 1.0};
    const int32_t re[3] = {0, 1, 0};
    const float rm[3] = {3.0e6f, 5.0e5f, 1.0e6f};
    const float z3[3] = {0, 0, 0};
    const float mx[3] = {1.2e7f, 2.0e6f, 4.0e6f};
    double y = -1, ypf = -1, g = -1, ov[3];
    int64_t h = -1;
    uint64_t c = 0;
    CHECK(orc_ara_run(1, 0, off, ev, 4, 1, lt, 2, el, eid, ro, et, re, rm, z3, z3, mx, 1, 0, 0,
                      NULL, 1, &y, &ypf, &g, &h, &c, ov) == 0);
    CHECK(y == 6.0e5 && ypf == 6.0e5 && g == 8.0e6 && h == 5);
    CHECK(ov[0] == 0.0 && ov[1] == 0.0 && ov[2] == 6.0e5);
}

static void random_portfolios(int su, int corr, int capped, int keying)
{
    enum { T = 40, NC = 16, MAXO = 12, NL = 2, NE = 5 };
    int64_t off[T + 1];
    int32_t ev[T * MAXO];
    off[0] = 0;
    for (int t = 0; t < T; ++t) {
        int n = (int)rnd(MAXO + 1);
        for (int k = 0; k < n; ++k) ev[off[t] + k] = (int32_t)rnd(NC);
        off[t + 1] = off[t] + n;
    }
    double lt[4 * NL];
    uint32_t prog[NL];
    for (int l = 0; l < NL; ++l) {
        lt[4 * l + 0] = 1e5 * rnd(20);
        lt[4 * l + 1] = l ? INFINITY : 1e7;
        lt[4 * l + 2] = 1e5 * rnd(50);
        lt[4 * l + 3] = l ? 3e7 : INFINITY;
        prog[l] = 7u + (uint32_t)l;
    }
    int32_t el[NE];
    uint32_t eid[NE];
    int64_t ro[NE + 1];
    double et[3 * NE];
    int32_t re[NE * NC];
    float rm[NE * NC], rsi[NE * NC], rsc[NE * NC], rmx[NE * NC];
    ro[0] = 0;
    for (int e = 0; e < NE; ++e) {
        el[e] = e % NL;
        eid[e] = 100u + (uint32_t)e;
        et[3 * e + 0] = 1e4 * rnd(10);
        et[3 * e + 1] = e == 1 ? INFINITY : 5e6;
        et[3 * e + 2] = e == 2 ? 0.5 : 1.0;
        int n = 0;
        for (int E = 0; E < NC; ++E) {
            if (rnd(3) == 0) continue;        /* distinct events, about 2/3 of the catalogue */
            int64_t r = ro[e] + n++;
            re[r] = E;
            rm[r] = (float)(1e5 * (1 + rnd(40)));
            rsi[r] = su ? (corr ? 0.25f : 0.5f) * rm[r] : 0.0f;
            rsc[r] = su && corr ? 0.25f * rm[r] : 0.0f;
            rmx[r] = 4.0f * rm[r];
            if (capped && (r % 3) == 0) rsi[r] = 3.0f * rm[r];
        }
        ro[e + 1] = ro[e] + n;
    }
    double ylt[NL * T], ypf[T], g[NL * T], ov[NL * T * MAXO];
    int64_t h[NL * T];
    uint64_t c[NL * T];
    CHECK(orc_ara_run(T, 1000, off, ev, NC, NL, lt, NE, el, eid, ro, et, re, rm, rsi, rsc, rmx,
                      150106326ull, su, keying, prog, 2, ylt, ypf, g, h, c, ov) == 0);
    for (int t = 0; t < T; ++t) {
        double s = 0.0;
        for (int l = 0; l < NL; ++l) {
            double y = ylt[l * T + t];
            CHECK(y >= 0.0 && y <= lt[4 * l + 3] && y <= g[l * T + t] + 1e-6);
            double d = 0.0;
            for (int64_t j = off[t]; j < off[t + 1]; ++j) d += ov[(int64_t)l * off[T] + j];
            CHECK(fabs(d - y) <= 1e-9 * (1.0 + y));
            s += y;
        }
        CHECK(fabs(s - ypf[t]) <= 1e-9 * (1.0 + s));
    }
    double rps[3] = {2.0, 10.0, 1000.0}, pml[3], tvar[3];
    CHECK(orc_pml_tvar(ypf, T, rps, 3, pml, tvar) == 0);
    for (int r = 0; r < 3; ++r) CHECK(pml[r] <= tvar[r] + 1e-6);
}

static void special_functions(void)
{
    const double shapes[][2] = {{2.75, 8.25}, {1.0, 1.0}, {0.5, 0.5}, {30.0, 70.0},
                                {5.0e-7, 1.5e-6}, {1e-3, 1e-3}, {3e-3, 1e-4}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
        for (uint32_t j = 1; j < (1u << 24); j += 1048573u * 2u) {
            double z = j / 16777216.0, zc = (16777216.0 - j) / 16777216.0, xc;
            double x = orc_betaincinv_pair(shapes[s][0], shapes[s][1], z, zc, &xc);
            CHECK(x >= 0.0 && x <= 1.0 && fabs(x + xc - 1.0) <= 1e-15);
            CHECK(orc_betainc(shapes[s][0], shapes[s][1], x) >= 0.0);
        }
    double a, b;
    orc_beta_fit(2.0, 2.0, 4.0, &a, &b);
    CHECK(a > 0 && b > 0 && a < 1e-5);
    CHECK(fabs(orc_norm_quantile(0.975) - 1.959963984540054) < 1e-14);
    CHECK(fabs(orc_norm_cdf(0.0) - 0.5) < 1e-16);
    const uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6};
    uint32_t o1[4], o2[4];
    orc_philox4x32_10(ctr, key, o1);
    orc_philox4x32_10(ctr, key, o2);
    CHECK(memcmp(o1, o2, sizeof o1) == 0);
}

int main(void)
{
    worked_example();
    for (int rep = 0; rep < 3; ++rep) {
        random_portfolios(0, 0, 0, 0);
        random_portfolios(1, 0, 0, 0);
        random_portfolios(1, 1, 0, 0);
        random_portfolios(1, 0, 1, 0);
        random_portfolios(1, 1, 0, 1);
    }
    special_functions();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: all checks held\n");
    return 0;
}
