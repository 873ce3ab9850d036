/*
 * ara_oracle.c -- plain, slow, FP64 CPU oracle for Aggregate Risk Analysis.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product path never does.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What it computes (B. Varghese, "The GPU vs Phi Debate: Risk Analytics Using
 * Many-Core Computing"):
 *   - Algorithm 1 (section 2.2): for every layer, trial and event occurrence
 *     (in stored, i.e. ascending-time, order) and every ELT of the layer:
 *     look the event up, apply the ELT financial terms, accumulate across
 *     ELTs; then the occurrence terms, then the aggregate terms on the
 *     cumulative sum; the last cumulative value is the trial's YLT entry.
 *   - Secondary uncertainty (section 3): combining sigma_I / sigma_C
 *     (section 3.2, five steps), the Beta moment fit with the sigma cap and
 *     Loss = max_l * InvCDF_beta(z; alpha, beta) (section 3.3), inserted after
 *     the lookup and before the ELT terms.
 *   - PML and TVaR from the YLT (section 2.3, named only).
 *
 * Readings where the paper is silent or garbled (each also listed in the
 * design notes of the repository):
 *   R1  ELT terms: l' = share * min(max(x - retention, 0), limit).
 *   R2  Aggregate terms act on the running sum S_k of occurrence losses, never
 *       fed back: A_k = min(max(S_k - AggR, 0), AggL); trial loss = A_last.
 *   R3  The uniform -> normal step of section 3.2 is the normal *quantile*.
 *   R4  Draws come from Philox4x32-10 (Salmon et al., SC'11): counter
 *       (k, i, elt_id, 0) for the independent draw u_I, (k, i, 0, 1) for the
 *       shared correlated draw u_C; key = (seed low, seed high); output word
 *       x0 mapped to u = ((x0 >> 8) | 1) * 2^-24.  k is the occurrence index
 *       inside the trial, i the absolute trial index.
 *       sigma_C = 0 -> z = u_I exactly; sigma_I = 0 -> z = u_C exactly.
 *   R5  sigma = sigma_I + sigma_C feeds the Beta (raw sum, as written).
 *   R6  Section 3.3 caps the standard deviation fed to the Beta fit just below
 *       sigma_beta_max without giving the margin: if sigma_beta >=
 *       sigma_beta_max use (1 - 1e-6) * sigma_beta_max.
 *   R7  sigma = 0 or secondary uncertainty off -> loss = mean, no draw.
 *   R8  PML(RP) = k-th largest trial loss, TVaR(RP) = mean of the k largest,
 *       with k = max(1, floor(N / RP)).
 *   R9  Both z and its complement 1 - z are carried, the complement computed
 *       directly (1 - u on the draw grid, Phi(-v) after the normal mix), so
 *       upper-tail quantiles keep full relative accuracy.
 *   R10 Optional keying that follows the input layout of section 3.1: the
 *       independent draw is z_(Prog,E), one per occurrence and program,
 *       counter (k, i, program_id, 2), shared by every ELT of the program's
 *       layers; the correlated draw is z_(E), a value held per XELT row for
 *       its event and the same in every occurrence, ELT and program, counter
 *       (E, 0, 0, 3).  (R4 is the default keying.)
 *
 * Numerics: Phi from erfc; Phi^-1 by bracketed Newton on that Phi; I_x(a,b)
 * by the continued fraction of DLMF 8.17.22 (modified Lentz) with the
 * symmetry I_x(a,b) = 1 - I_{1-x}(b,a) and an lgamma prefactor; I^-1 by
 * bisection-safeguarded Newton to ~1e-15 relative.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  One round maps (c0,c1,c2,c3) with key (k0,k1)  */
/* to (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0)); the key is   */
/* bumped by the Weyl constants between rounds.                               */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u = ((w >> 8) | 1) * 2^-24: an odd multiple of 2^-24 in (0, 1). */
double orc_u01(uint32_t w)
{
    return (double)((w >> 8) | 1u) * (1.0 / 16777216.0);
}

static double draw_u(uint32_t k, uint32_t i, uint32_t c2, uint32_t stream, uint64_t seed)
{
    uint32_t ctr[4] = { k, i, c2, stream };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return orc_u01(out[0]);
}

/* ------------------------------------------------------------------------ */
/* Normal distribution                                                        */
/* ------------------------------------------------------------------------ */
double orc_norm_cdf(double x)
{
    return 0.5 * erfc(-x / sqrt(2.0));
}

static double norm_pdf(double x)
{
    return exp(-0.5 * x * x) / sqrt(2.0 * M_PI);
}

/* Phi^-1(p) for p in (0, 1): bisection to a short bracket, then Newton on
 * Phi(x) - p with the bracket kept as a safeguard.  The lower half is solved
 * directly; the upper half through Phi^-1(p) = -Phi^-1(1 - p). */
double orc_norm_quantile(double p)
{
    if (!(p > 0.0)) return -INFINITY;
    if (!(p < 1.0)) return INFINITY;
    if (p > 0.5) return -orc_norm_quantile(1.0 - p);
    if (p == 0.5) return 0.0;
    double lo = -40.0, hi = 0.0, x = -1.0;
    for (int it = 0; it < 60; ++it) {          /* bisection to width < 1e-3 */
        x = 0.5 * (lo + hi);
        if (orc_norm_cdf(x) < p) lo = x; else hi = x;
        if (hi - lo < 1e-3) break;
    }
    x = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        double f = orc_norm_cdf(x) - p;
        if (f < 0) lo = x; else hi = x;
        double xn = x - f / norm_pdf(x);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-16 * fabs(xn)) { x = xn; break; }
        x = xn;
    }
    return x;
}

/* ------------------------------------------------------------------------ */
/* Regularized incomplete beta I_x(a, b) and its inverse                      */
/* ------------------------------------------------------------------------ */
static double log_beta(double a, double b)
{
    return lgamma(a) + lgamma(b) - lgamma(a + b);
}

/* Continued fraction of DLMF 8.17.22 by the modified Lentz method:
 *   I_x(a,b) = x^a (1-x)^b / (a B(a,b)) * 1/(1+ d1/(1+ d2/(1+ ...)))
 *   d_{2m+1} = -(a+m)(a+b+m) x / ((a+2m)(a+2m+1))
 *   d_{2m}   =  m (b-m) x / ((a+2m-1)(a+2m))
 * The modified Lentz recurrence below evaluates K = 1 + d1/(1 + d2/(...))
 * (b0 = 1, a_n = d_n, b_n = 1); the function returns 1/K. */
static double beta_cf(double a, double b, double x)
{
    const double tiny = 1e-300;
    double f = 1.0, C = 1.0, D = 0.0;
    for (int n = 1; n <= 20000; ++n) {
        int m = n / 2;
        double d;
        if (n & 1)
            d = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
        else
            d = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
        D = 1.0 + d * D;
        if (fabs(D) < tiny) D = tiny;
        C = 1.0 + d / C;
        if (fabs(C) < tiny) C = tiny;
        D = 1.0 / D;
        double delta = C * D;
        f *= delta;
        if (fabs(delta - 1.0) < 1e-16) break;
    }
    /* f has converged to K = 1 + d1/(1 + d2/(1 + ...)); the fraction in
     * DLMF 8.17.22 is 1/K. */
    return 1.0 / f;
}

/* I_x(a,b) and 1 - I_x(a,b), each computed without cancellation on its own
 * side of the switch point x = (a+1)/(a+b+2). */
void orc_betainc_pair(double a, double b, double x, double *I, double *Ic)
{
    if (x <= 0.0) { *I = 0.0; *Ic = 1.0; return; }
    if (x >= 1.0) { *I = 1.0; *Ic = 0.0; return; }
    double lnfront = a * log(x) + b * log1p(-x) - log_beta(a, b);
    if (x < (a + 1.0) / (a + b + 2.0)) {
        double v = exp(lnfront) * beta_cf(a, b, x) / a;
        *I = v; *Ic = 1.0 - v;
    } else {
        double v = exp(lnfront) * beta_cf(b, a, 1.0 - x) / b;
        *Ic = v; *I = 1.0 - v;
    }
}

double orc_betainc(double a, double b, double x)
{
    double I, Ic;
    orc_betainc_pair(a, b, x, &I, &Ic);
    return I;
}

/* Solve I_x(a,b) = z for x, when the root lies in (0, 1/2]; zc = 1 - z.
 * Newton's method on the logarithm of the smaller side -- ln I_x - ln z when
 * z <= 1/2, ln(1 - I_x) - ln zc otherwise -- so the residual never cancels and
 * stays well scaled in the tails; the slopes are f/I_x and -f/(1 - I_x), f
 * the Beta density.  The bracket [lo, hi], shrunk by every evaluation of the
 * monotone I_x, safeguards it: a step leaving the bracket is replaced by
 * bisection. */
static double betainc_solve_lower(double a, double b, double z, double zc)
{
    if (!(z > 0.0)) return 0.0;
    int use_lower = z <= zc;
    double lb = log_beta(a, b);
    double lo = 0.0, hi = 0.5;
    /* leading term of the small-x expansion I_x ~ x^a / (a B(a,b)) */
    double x = exp((log(z) + log(a) + lb) / a);
    if (!(x > 0.0)) return 0.0;               /* below the smallest double */
    if (!(x < 0.5)) x = 0.25;
    for (int it = 0; it < 5000; ++it) {
        double I, Ic;
        orc_betainc_pair(a, b, x, &I, &Ic);
        double dens = exp((a - 1.0) * log(x) + (b - 1.0) * log1p(-x) - lb);
        double step;
        if (use_lower) {
            if (I == z) return x;
            if (I < z) lo = x; else hi = x;
            step = -log(I / z) * I / dens;
        } else {
            if (Ic == zc) return x;
            if (Ic > zc) lo = x; else hi = x;
            step = log(Ic / zc) * Ic / dens;
        }
        double xn = x + step;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 2e-16 * xn) return xn;
        x = xn;
    }
    return x;
}

/* x with I_x(a,b) = z, given z and its complement zc = 1 - z.  Returns x and
 * writes 1 - x to *xc.  The root is solved for on the side where it is at
 * most 1/2 (x <= 1/2 exactly when z <= I_{1/2}(a,b)); the other side follows
 * from I_{1-x}(b,a) = 1 - z, so both x and 1 - x keep full relative
 * precision, also for near-Bernoulli shapes whose roots sit at 1e-100. */
double orc_betaincinv_pair(double a, double b, double z, double zc, double *xc)
{
    double x, y, Ih, Ihc;
    orc_betainc_pair(a, b, 0.5, &Ih, &Ihc);
    int root_low = (z <= zc) ? (z <= Ih) : (zc >= Ihc);
    if (root_low) {
        x = betainc_solve_lower(a, b, z, zc);
        y = 1.0 - x;
    } else {
        y = betainc_solve_lower(b, a, zc, z);  /* I_{1-x}(b,a) = 1 - z */
        x = 1.0 - y;
    }
    if (xc) *xc = y;
    return x;
}

double orc_betaincinv(double a, double b, double z)
{
    return orc_betaincinv_pair(a, b, z, 1.0 - z, NULL);
}

/* Beta moment fit of section 3.3: mu_b = mu/max, sigma_b = sigma/max,
 * sigma_b_max = sqrt(mu_b (1 - mu_b)), capped per R6,
 * alpha = mu_b ((sigma_b_max/sigma_b)^2 - 1), beta = (1 - mu_b)(...). */
void orc_beta_fit(double mu, double sigma, double max_l, double *alpha, double *beta)
{
    double mu_b = mu / max_l;
    double s_b = sigma / max_l;
    double s_bmax = sqrt(mu_b * (1.0 - mu_b));
    if (s_b >= s_bmax) s_b = (1.0 - 1e-6) * s_bmax;
    double r = s_bmax / s_b;
    double kappa = r * r - 1.0;
    *alpha = mu_b * kappa;
    *beta = (1.0 - mu_b) * kappa;
}

/* Section 3.2: combine the two uniforms into z (and its complement). */
static void combine_sigma(double u_pe, double u_e, double s_i, double s_c,
                          double *z, double *zc)
{
    double sigma = s_i + s_c;                          /* step i   */
    double v_pe = orc_norm_quantile(u_pe);              /* step ii  */
    double v_e = orc_norm_quantile(u_e);
    double wi = s_i / sigma, wc = s_c / sigma;
    double lc = v_pe * wi + v_e * wc;                   /* step iii */
    double v = lc / sqrt(wi * wi + wc * wc);            /* step iv  */
    *z = orc_norm_cdf(v);                               /* step v   */
    *zc = orc_norm_cdf(-v);
}

/* Loss of one ELT row hit by occurrence k (event E) of trial i (secondary
 * uncertainty on), section 3: draw, combine, fit, invert, scale by max_l.
 * keying 0: R4; keying 1: R10 (program = the layer's program id). */
double orc_su_loss_keyed(double mu, double s_i, double s_c, double max_l,
                         uint32_t k, uint32_t i, uint32_t elt_id, uint32_t program,
                         uint32_t event, int32_t keying, uint64_t seed)
{
    double sigma = s_i + s_c;
    if (sigma == 0.0) return mu;                        /* R7 */
    /* the two uniforms of section 3.1 (i) and (ii) */
    uint32_t ci[4] = {k, i, elt_id, 0}, cc[4] = {k, i, 0, 1};
    if (keying == 1) {
        ci[2] = program; ci[3] = 2;
        cc[0] = event; cc[1] = 0; cc[2] = 0; cc[3] = 3;
    }
    double z, zc;
    if (s_c == 0.0) {
        double u = draw_u(ci[0], ci[1], ci[2], ci[3], seed);
        z = u; zc = 1.0 - u;
    } else if (s_i == 0.0) {
        double u = draw_u(cc[0], cc[1], cc[2], cc[3], seed);
        z = u; zc = 1.0 - u;
    } else {
        double u_pe = draw_u(ci[0], ci[1], ci[2], ci[3], seed);
        double u_e = draw_u(cc[0], cc[1], cc[2], cc[3], seed);
        combine_sigma(u_pe, u_e, s_i, s_c, &z, &zc);
    }
    double alpha, beta;
    orc_beta_fit(mu, sigma, max_l, &alpha, &beta);
    double x = orc_betaincinv_pair(alpha, beta, z, zc, NULL);
    return max_l * x;
}

double orc_su_loss(double mu, double s_i, double s_c, double max_l,
                   uint32_t k, uint32_t i, uint32_t elt_id, uint64_t seed)
{
    return orc_su_loss_keyed(mu, s_i, s_c, max_l, k, i, elt_id, 0, 0, 0, seed);
}

/* ------------------------------------------------------------------------ */
/* Aggregate Risk Analysis, Algorithm 1 with secondary uncertainty            */
/* ------------------------------------------------------------------------ */
static double clamp_terms(double x, double retention, double limit)
{
    return fmin(fmax(x - retention, 0.0), limit);
}

/* Inputs, all host arrays:
 *   YET trials [0, n_trials): offsets[n_trials+1] into event_ids (offsets[0]
 *   need not be 0); absolute trial index of trial t is trial_base + t.
 *   ELTs e = 0..n_elt-1: elt_layer[e] (layer it belongs to; ELTs of a layer
 *   are listed in their order), elt_id[e], elt_row_off[n_elt+1] into the row
 *   arrays, elt_terms[3e..3e+2] = (retention, limit, share).
 *   layer_terms[4l..4l+3] = (OccR, OccL, AggR, AggL); layer_program[l] (may
 *   be NULL: all 0) keys z_(Prog,E) when keying = 1 (R10).
 * Outputs (each may be NULL except ylt): ylt[l*n_trials + t] trial loss of
 *   layer l; ylt_pf[t] = sum over layers; gross[l*n_trials+t] = sum_k X_k;
 *   hits / hit_chk[l*n_trials+t]: number of non-zero lookups and the checksum
 *   sum over hits of (k+1)*2654435761 + elt_id (mod 2^64);
 *   occ_view[l*n_occ_total + (offsets[t]-offsets[0]) + k]: the per-occurrence
 *   increment d_k = A_k - A_{k-1} of the aggregate terms.
 * Returns 0, or -1 on a bad argument (an event id outside the catalogue). */
int orc_ara_run(int64_t n_trials, int64_t trial_base, const int64_t *offsets,
                const int32_t *event_ids, int32_t n_catalogue,
                int32_t n_layers, const double *layer_terms,
                int32_t n_elt, const int32_t *elt_layer, const uint32_t *elt_id,
                const int64_t *elt_row_off, const double *elt_terms,
                const int32_t *row_event, const float *row_mean,
                const float *row_sigma_i, const float *row_sigma_c,
                const float *row_max, uint64_t seed, int32_t su_enabled,
                int32_t keying, const uint32_t *layer_program, int32_t n_threads,
                double *ylt, double *ylt_pf, double *gross, int64_t *hits,
                uint64_t *hit_chk, double *occ_view)
{
    /* Direct-access tables (section 4.2): for each ELT a catalogue-sized array
     * holding the row index of each event, or -1 where the loss is zero. */
    int64_t *dat = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_elt * (size_t)n_catalogue);
    if (!dat) return -2;
    for (int64_t j = 0; j < (int64_t)n_elt * n_catalogue; ++j) dat[j] = -1;
    for (int32_t e = 0; e < n_elt; ++e)
        for (int64_t r = elt_row_off[e]; r < elt_row_off[e + 1]; ++r) {
            int32_t ev = row_event[r];
            if (ev < 0 || ev >= n_catalogue) { free(dat); return -1; }
            dat[(int64_t)e * n_catalogue + ev] = r;
        }
    for (int64_t t = 0; t < n_trials; ++t)
        for (int64_t j = offsets[t]; j < offsets[t + 1]; ++j)
            if (event_ids[j] < 0 || event_ids[j] >= n_catalogue) { free(dat); return -1; }

    int64_t occ_total = offsets[n_trials] - offsets[0];
    if (ylt_pf)
        for (int64_t t = 0; t < n_trials; ++t) ylt_pf[t] = 0.0;

#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    /* Every layer is priced on every trial independently (section 2.2); a
     * trial's occurrences are visited in stored (ascending time) order and,
     * for each, every ELT of the layer in its listed order. */
    for (int32_t l = 0; l < n_layers; ++l) {
        double occR = layer_terms[4 * l + 0], occL = layer_terms[4 * l + 1];
        double aggR = layer_terms[4 * l + 2], aggL = layer_terms[4 * l + 3];
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < n_trials; ++t) {
            uint32_t i_abs = (uint32_t)(trial_base + t);
            double S = 0.0, A_prev = 0.0, G = 0.0;
            int64_t nh = 0;
            uint64_t chk = 0;
            int64_t base = offsets[t];
            for (int64_t j = base; j < offsets[t + 1]; ++j) {
                uint32_t k = (uint32_t)(j - base);
                int32_t E = event_ids[j];
                double X = 0.0;
                for (int32_t e = 0; e < n_elt; ++e) {
                    if (elt_layer[e] != l) continue;
                    /* direct-access table: -1 marks an event the ELT does not cover */
                    int64_t r = dat[(int64_t)e * n_catalogue + E];
                    if (r < 0) continue;
                    ++nh;
                    chk += (uint64_t)(k + 1) * 2654435761ull + (uint64_t)elt_id[e];
                    double mu = row_mean[r];
                    double loss;
                    if (!su_enabled) loss = mu;
                    else loss = orc_su_loss_keyed(mu, row_sigma_i[r], row_sigma_c[r],
                                                  row_max[r], k, i_abs, elt_id[e],
                                                  layer_program ? layer_program[l] : 0u,
                                                  (uint32_t)E, keying, seed);
                    double lp = elt_terms[3 * e + 2] *
                                clamp_terms(loss, elt_terms[3 * e + 0], elt_terms[3 * e + 1]);
                    X += lp;                       /* event loss X_k over the layer's ELTs */
                }
                G += X;
                double O = clamp_terms(X, occR, occL);     /* occurrence terms on X_k */
                S += O;                                    /* running sum, never clamped */
                double A = clamp_terms(S, aggR, aggL);     /* aggregate terms on S_k (R2) */
                if (occ_view) occ_view[(int64_t)l * occ_total + (j - offsets[0])] = A - A_prev;
                A_prev = A;
            }
            double Y = A_prev;
            ylt[(int64_t)l * n_trials + t] = Y;
            if (gross) gross[(int64_t)l * n_trials + t] = G;
            if (hits) hits[(int64_t)l * n_trials + t] = nh;
            if (hit_chk) hit_chk[(int64_t)l * n_trials + t] = chk;
        }
        if (ylt_pf)
            for (int64_t t = 0; t < n_trials; ++t) ylt_pf[t] += ylt[(int64_t)l * n_trials + t];
    }
    free(dat);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* PML and TVaR (reading R8), by full sort                                     */
/* ------------------------------------------------------------------------ */
static int cmp_desc(const void *pa, const void *pb)
{
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a < b) - (a > b);
}

int orc_pml_tvar(const double *ylt, int64_t n, const double *rps, int32_t n_rp,
                 double *pml, double *tvar)
{
    if (n <= 0) return -1;
    double *s = (double *)malloc(sizeof(double) * (size_t)n);
    if (!s) return -2;
    memcpy(s, ylt, sizeof(double) * (size_t)n);
    qsort(s, (size_t)n, sizeof(double), cmp_desc);
    for (int32_t r = 0; r < n_rp; ++r) {
        int64_t k = (int64_t)floor((double)n / rps[r]);
        if (k < 1) k = 1;
        if (k > n) k = n;
        pml[r] = s[k - 1];
        long double acc = 0.0L;
        for (int64_t j = 0; j < k; ++j) acc += (long double)s[j];
        tvar[r] = (double)(acc / (long double)k);
    }
    free(s);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Array helpers for the test harness (loops over the scalar functions).      */
/* ------------------------------------------------------------------------ */
void orc_philox_batch(int64_t n, const uint32_t *ctrs, const uint32_t key[2], uint32_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) orc_philox4x32_10(ctrs + 4 * j, key, out + 4 * j);
}

void orc_draw_u_batch(int64_t n, const uint32_t *ctrs, uint64_t seed, double *u)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        u[j] = draw_u(ctrs[4 * j], ctrs[4 * j + 1], ctrs[4 * j + 2], ctrs[4 * j + 3], seed);
}

void orc_betaincinv_batch(int64_t n, const double *a, const double *b, const double *z,
                          const double *zc, double *x, double *xc)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        double y;
        x[j] = orc_betaincinv_pair(a[j], b[j], z[j], zc[j], &y);
        if (xc) xc[j] = y;
    }
}

void orc_betainc_batch(int64_t n, const double *a, const double *b, const double *x,
                       double *I, double *Ic)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        double v, w;
        orc_betainc_pair(a[j], b[j], x[j], &v, &w);
        I[j] = v;
        if (Ic) Ic[j] = w;
    }
}

void orc_norm_batch(int64_t n, const double *in, double *cdf, double *quantile)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        if (cdf) cdf[j] = orc_norm_cdf(in[j]);
        if (quantile) quantile[j] = orc_norm_quantile(in[j]);
    }
}

void orc_su_loss_batch(int64_t n, const double *mu, const double *s_i, const double *s_c,
                       const double *max_l, const uint32_t *k, const uint32_t *i,
                       const uint32_t *elt_id, uint64_t seed, double *loss)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        loss[j] = orc_su_loss(mu[j], s_i[j], s_c[j], max_l[j], k[j], i[j], elt_id[j], seed);
}
