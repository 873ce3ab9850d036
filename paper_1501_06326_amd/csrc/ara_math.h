// ara_math.h -- device arithmetic of secondary uncertainty (section 3 of the
// paper): Philox4x32-10 draws, the normal mix of section 3.2 and the inverse
// regularized incomplete beta of section 3.3, in an FP32 bulk form and an
// FP64 form for the tails and for shapes the FP32 form does not cover.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ara_internal.h"

namespace ara {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The ten round keys are
// the same for every draw of a run, so the host expands them once
// (PhiloxKeys) and the device only runs the rounds.
// ---------------------------------------------------------------------------
struct PhiloxKeys {
    uint32_t k0, k1;           // the key; round r uses (k0 + r W0, k1 + r W1)
};

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

inline PhiloxKeys philox_keys(uint64_t seed) {
    PhiloxKeys k;
    k.k0 = (uint32_t)seed;
    k.k1 = (uint32_t)(seed >> 32);
    return k;
}

// The key is wave-uniform, so its schedule runs on the scalar unit.
__device__ __forceinline__ uint4 philox10(uint4 c, const PhiloxKeys &k) {
    uint32_t k0 = k.k0, k1 = k.k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)c.x;
        uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)c.z;
        uint4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return c;
}

// Word 0 only: the last round's x output needs only the product M1 * c.z.
__device__ __forceinline__ uint32_t philox10_x0(uint4 c, const PhiloxKeys &k) {
    uint32_t k0 = k.k0, k1 = k.k1;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)c.x;
        uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)c.z;
        uint4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return __umulhi(kPhiloxM1, c.z) ^ c.y ^ k0;
}

// Odd multiple of 2^-24: u = ((w >> 8) | 1) * 2^-24, so 1 - u is exact too.
// Returns the 24-bit odd integer j; u = j * 2^-24.
__device__ __forceinline__ uint32_t u24(uint32_t w) { return (w >> 8) | 1u; }

// ---------------------------------------------------------------------------
// FP32 building blocks
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

// Reciprocal with one Newton step (about 0.5 ulp): cheaper than an IEEE
// division where the last half ulp does not matter.
__device__ __forceinline__ float rcp_nr(float y) {
    const float r = rcp_f(y);
    return r * fmaf(-y, r, 2.0f);
}

// log2(1 - x) for 0 <= x < 1: w = 1 - x rounds, but its rounding error
// e = (1 - w) - x is exact (Fast2Sum, |1| >= |x|), and
// log2(1 - x) = log2(w) + log2(1 + e/w) ~ log2(w) + (e/w) log2(e).
__device__ __forceinline__ float log2_1m(float x, float w) {
    const float e = (1.0f - w) - x;
    return fmaf(e * rcp_f(w), 1.4426950408889634f, __log2f(w));
}

// Continued fraction of DLMF 8.17.22: I_x(a, b) = x^a (1-x)^b / (a B(a,b)) / K
// with K = 1 + d1/(1 + d2/(1 + ...)),
//   d_{2m+1} = -(a+m)(a+b+m) x / ((a+2m)(a+2m+1)),
//   d_{2m}   =  m(b-m) x / ((a+2m-1)(a+2m)).
// Evaluated backward from term n (more accurate in FP32 than the forward
// recurrence) without divisions: with d_j = p_j / q_j and K_j = N_j / D_j,
// N_j = q_j N_{j+1} + p_j D_{j+1}, D_j = q_j N_{j+1}.  Terms go in pairs
// (2m, 2m-1); n (even) comes from the row (enough terms at the slowest
// point of the branch, see cf_terms); lanes with fewer terms than the batch
// maximum nmax (even, wave-uniform) leave their (N, D) at the start value
// until their first term, a select that is skipped when every lane needs
// nmax terms.  Rescaled every pair.  Returns N, D.
__device__ __forceinline__ void beta_cf32(float a, float b, float x, int n, int nmax, float *Nout,
                                          float *Dout) {
    float N = 1.0f, D = 1.0f;
    const float am1 = a - 1.0f, apbm1 = (a + b) - 1.0f;
    // one pair of terms (2m, 2m-1), rescaled to N = 1
    auto pair = [&](float fm, float *Dn) {
        // even term 2m: p = m (b - m) x, q = (a + 2m - 1)(a + 2m) = te (te + 1)
        const float te = fmaf(2.0f, fm, am1);
        const float qe = fmaf(te, te, te);
        const float pe = fm * (b - fm) * x;
        // odd term 2m-1: p = -(a+m-1)(a+b+m-1) x, q = (a+2m-2)(a+2m-1) = (te - 1) te
        const float qo = fmaf(te, te, -te);
        const float po = -(am1 + fm) * (apbm1 + fm) * x;
        const float N1 = fmaf(qe, N, pe * D), D1 = qe * N;
        const float N2 = fmaf(qo, N1, po * D1), D2 = qo * N1;
        *Dn = D2 * rcp_f(N2);
    };
    float fm = (float)(nmax >> 1);           // exact small integer, stepped down exactly
    if (__all(n >= nmax)) {
        // every lane takes every term (the usual case: one shape per batch)
        for (int m = nmax >> 1; m >= 1; --m, fm -= 1.0f) pair(fm, &D);
    } else {
        for (int m = nmax >> 1; m >= 1; --m, fm -= 1.0f) {
            float Dn;
            pair(fm, &Dn);
            const bool on = 2 * m <= n;
            N = on ? 1.0f : N;
            D = on ? Dn : D;
        }
    }
    *Nout = N;
    *Dout = D;
}

// Terms of the continued fraction that FP32 needs (truncation below 1e-8
// relative) at the slowest point of its branch, x = (a+1)/(a+b+2); it
// converges faster for smaller x.  Evaluated in FP64 at load time; 0 when
// more than 62 terms would be needed.  The reference takes 200 terms: where
// 62 terms reach 1e-8 the fraction converges at least as fast as 0.75^n, so
// 200 terms are exact to FP64 rounding.
__device__ inline int cf_terms(double a, double b) {
    const double x = (a + 1.0) / (a + b + 2.0);
    auto eval = [&](int n) {
        double K = 1.0;
        for (int j = n; j >= 1; --j) {
            const int m = j >> 1;
            // d_j = p / q; K <- 1 + d_j / K with one division
            const double p = (j & 1) ? -(a + m) * (a + b + m) * x : m * (b - m) * x;
            const double q = (j & 1) ? (a + 2.0 * m) * (a + 2.0 * m + 1.0)
                                     : (a + 2.0 * m - 1.0) * (a + 2.0 * m);
            K = 1.0 + p / (q * K);
        }
        return 1.0 / K;
    };
    const double ref = eval(200);
    for (int n = 2; n <= 62; n += 2)
        if (fabs(eval(n) / ref - 1.0) < 1e-8) return n;
    return 0;
}

// Initial guess: Abramowitz & Stegun 26.2.22 for the upper-tail normal
// deviate y of the smaller tail probability, then A&S 26.5.22 for the Beta
// quantile (valid for a, b > 1/2; used here for a, b >= 1).
__device__ __forceinline__ float beta_guess32(float a, float b, float z, float zc) {
    // only a starting point: approximate reciprocals are enough
    const bool lowz = z < 0.5f;
    const float pp = lowz ? z : zc;
    const float t = sqrtf(-2.0f * __logf(pp));
    float y = t - (2.30753f + 0.27061f * t) * rcp_f(1.0f + t * (0.99229f + 0.04481f * t));
    if (!lowz) y = -y;                       // y = Phi^-1(1 - z)
    const float lam = (y * y - 3.0f) * (1.0f / 6.0f);
    const float ra = rcp_f(2.0f * a - 1.0f), rb = rcp_f(2.0f * b - 1.0f);
    const float rh = 0.5f * (ra + rb);       // 1 / h, h = 2 / (ra + rb)
    const float w = y * sqrtf(rcp_f(rh) + lam) * rh -
                    (rb - ra) * (lam + 5.0f / 6.0f - (2.0f / 3.0f) * rh);
    return a * rcp_f(a + b * __expf(2.0f * w));
}

// Starting point from a shape table (the layout is described with
// kShapeSlots): the logit of the quantile, interpolated linearly in
// t = sqrt(-2 ln p) between the two table points around the draw, on the
// table half of its z.  z is an odd multiple of 2^-24, so p = min(z, 1 - z)
// lies in [2^-24, 1/2) and t inside the table's range.
__device__ __forceinline__ float shape_guess_logit(const float *tab, float z, float zc) {
    const bool upper = z > 0.5f;
    const float p = upper ? zc : z;
    const float t = sqrtf(-2.0f * __logf(p));
    const float inv_h = (float)((kShapeK - 1) / (kShapeTHi - kShapeTLo));
    const float u = fminf(fmaxf((t - (float)kShapeTLo) * inv_h, 0.0f), (float)(kShapeK - 1));
    const int i = min((int)u, kShapeK - 2);
    const float f = u - (float)i;
    const float *T = tab + (upper ? kShapeK : 0) + i;
    const float l0 = T[0], l1 = T[1];
    return fmaf(f, l1 - l0, l0);
}

// I_x(a,b) (*I) and 1 - I_x(a,b) (*Ic), each on the side where it is
// accurate, and the prefactor x^a (1-x)^b / B(a,b) (*front; the density is
// front / (x (1-x))); lnb2 = log2 B(a, b); na / nb the continued-fraction
// terms of the (a, b) and (b, a) branches; nmax the wave-uniform bound of both.
__device__ __forceinline__ void beta_inc32(float a, float b, float lnb2, int na, int nb, int nmax,
                                           float x, float *I, float *Ic, float *front_out) {
    const float w = 1.0f - x;
    const float e2 = fmaf(a, __log2f(x), fmaf(b, log2_1m(x, w), -lnb2));
    const float front = exp2f(e2);
    *front_out = front;
    const bool direct = x * (a + b + 2.0f) < a + 1.0f;
    // one loop for both branches: (a, b, x) directly, else (b, a, 1 - x)
    const float A = direct ? a : b, B = direct ? b : a, X = direct ? x : w;
    float N, D;
    beta_cf32(A, B, X, direct ? na : nb, nmax, &N, &D);
    const float v = front * D * rcp_nr(N * A);
    *I = direct ? v : 1.0f - v;
    *Ic = direct ? 1.0f - v : v;
}

// FP32 quantile x = I^-1(z; a, b) given z and zc = 1 - z (both exact), for
// shapes inside the FP32 domain (kF32MinShape <= a, b <= kF32MaxShape).
// Halley iterations on the side where the root is at most ~1/2 (mirroring
// through I_{1-x}(b,a) = 1 - z otherwise), with the residual taken on the
// side of the smaller of z, zc so it never cancels.  The first iteration
// evaluates the continued fraction with about half its terms (the guess is
// only good to ~1e-2, so a residual good to ~1e-4 serves that step); every
// later one uses all of them.  The step sizes use reciprocals (they only set
// the speed, the residual sets the root): with f the density and r the
// residual, u = r / f = r x (1-x) / front and u (log f)' = r ((a-1)(1-x) -
// (b-1) x) / front share one reciprocal.  Stops when every lane's last
// full-accuracy step was below 2^-10 of the root (Halley: the next error ~
// step^3); a lane keeps the iterate of its own first such step, so its
// result does not depend on how many iterations the wavefront runs.  Returns
// false in *ok if it did not converge (the caller then uses the FP64 path).
// With a shape table (tab, the row's slot; null without) the start comes
// from the table instead, within ~2.2e-4 of the root: the first iteration
// then takes every term and its step already decides convergence, so one
// Halley step is the usual cost.  Whether a lane has a table depends on its
// row only, so its result still does not depend on the lanes beside it.
__device__ __forceinline__ float beta_quantile32(float a, float b, float lnb2, int na, int nb,
                                                 float z, float zc, const float *tab, bool *ok) {
    const bool full0 = tab != nullptr;
    float x0;
    bool mirror;
    if (full0) {
        // the small side of the root straight from the logit L = ln(x/(1-x)):
        // x = 1/(1+e^-L) = 1/(1+e^|L|) when L <= 0, else 1 - x = 1/(1+e^L)
        const float L = shape_guess_logit(tab, z, zc);
        mirror = L > 0.0f;
        x0 = rcp_f(1.0f + __expf(fabsf(L)));
    } else {
        x0 = beta_guess32(a, b, z, zc);
        mirror = x0 > 0.5f;
        if (mirror) x0 = 1.0f - x0;
    }
    float A = a, B = b, Z = z, ZC = zc;
    int NA = na, NB = nb;
    if (mirror) {
        A = b; B = a; Z = zc; ZC = z; NA = nb; NB = na;
    }
    // bound of both branches' term counts over the active lanes only (a
    // shuffle would also read the registers of inactive lanes): bitwise
    // maximum by ballots, counts are below 64
    const int nl = max(na, nb);
    int nmax = 0;
#pragma unroll
    for (int bit = 32; bit >= 1; bit >>= 1)
        if (__any(nl >= (nmax | bit))) nmax |= bit;
    const int nhalf = max(2, ((nmax >> 1) + 1) & ~1);
    // this lane's own half count (the wave's bounds only size the loops, so a
    // lane's result does not depend on the lanes beside it)
    const int nh = max(2, ((nl >> 1) + 1) & ~1);
    float x = fminf(fmaxf(x0, 1e-30f), 0.75f);
    const bool lower = Z <= 0.5f;
    const float am1 = A - 1.0f, bm1 = B - 1.0f;
    bool conv = false;
    float xf = x;          // the lane's answer: its iterate at its own first convergence
    const int nt0 = __any(full0) ? nmax : nhalf;
    for (int it = 0; it < 6; ++it) {
        const int nt = it == 0 ? nt0 : nmax;
        const int nown = (it == 0 && !full0) ? nh : nmax;
        float I, Ic, front;
        beta_inc32(A, B, lnb2, min(NA, nown), min(NB, nown), nt, x, &I, &Ic, &front);
        const float r = lower ? (I - Z) : (ZC - Ic);
        const float w = 1.0f - x;
        const float rf = r * rcp_f(front);
        const float u = rf * (x * w);
        const float uh = rf * fmaf(am1, w, -bm1 * x);
        const float t = u * rcp_f(1.0f - 0.5f * fminf(1.0f, uh));
        float xn = x - t;
        if (!(xn > 0.0f)) xn = 0.5f * x;
        if (!(xn < 1.0f)) xn = 0.5f * (x + 1.0f);
        if (!conv) {
            xf = xn;
            conv = (it > 0 || full0) && fabsf(xn - x) <= 9.765625e-4f * xn;
        }
        x = xn;
        if (__all(conv)) break;
    }
    *ok = conv && isfinite(xf);
    return mirror ? 1.0f - xf : xf;
}

// ---------------------------------------------------------------------------
// FP64 path (tails, shapes outside the FP32 domain, FP32 non-convergence).
// ---------------------------------------------------------------------------
__device__ inline double beta_cf64(double a, double b, double x) {
    double Am2 = 1.0, Bm2 = 0.0, Am1 = 1.0, Bm1 = 1.0, qprev = 1.0, Kprev = 1.0, K = 1.0;
    const double apb = a + b;
    for (int m = 0; m < 4000; ++m) {
        const double fm = (double)m;
        const double t0 = a + 2.0 * fm;
        const double qo = t0 * (t0 + 1.0);
        const double ao = qprev * (-(a + fm) * (apb + fm) * x);
        const double A1 = qo * Am1 + ao * Am2;
        const double B1 = qo * Bm1 + ao * Bm2;
        const double qe = (t0 + 1.0) * (t0 + 2.0);
        const double ae = qo * ((fm + 1.0) * (b - fm - 1.0) * x);
        const double A2 = qe * A1 + ae * Am1;
        const double B2 = qe * B1 + ae * Bm1;
        qprev = qe;
        const double s = 1.0 / B2;
        Am2 = A1 * s;
        Bm2 = B1 * s;
        Am1 = A2 * s;
        Bm1 = 1.0;
        K = Am1;
        if (fabs(K - Kprev) <= 1e-16 * fabs(K)) break;
        Kprev = K;
    }
    return 1.0 / K;
}

__device__ inline void beta_inc64(double a, double b, double lnb, double x, double *I, double *Ic,
                                  double *logdens) {
    const double lx = log(x), l1x = log1p(-x);
    const double e = a * lx + b * l1x - lnb;
    *logdens = e - lx - l1x;
    if (x * (a + b + 2.0) < a + 1.0) {
        const double P = exp(e) * beta_cf64(a, b, x) / a;
        *I = P;
        *Ic = 1.0 - P;
    } else {
        const double Q = exp(e) * beta_cf64(b, a, 1.0 - x) / b;
        *Ic = Q;
        *I = 1.0 - Q;
    }
}

// Solve I_x(a,b) = z for a root known to lie in (0, hi0]; Halley steps
// bracketed by [lo, hi] (every evaluation of the increasing I_x shrinks the
// bracket); a step leaving the bracket falls back to bisection, geometric
// while the bracket spans decades.  Returns false in *ok on failure.
__device__ inline double beta_solve64(double a, double b, double lnb, double z, double zc,
                                      double x, double hi0, int max_iter, bool *ok) {
    const bool lower = z <= zc;
    double lo = 0.0, hi = hi0;
    if (!(x > 0.0 && x < hi)) x = 0.5 * hi;
    *ok = false;
    for (int it = 0; it < max_iter; ++it) {
        double I, Ic, ld;
        beta_inc64(a, b, lnb, x, &I, &Ic, &ld);
        const double r = lower ? (I - z) : (zc - Ic);
        if (r == 0.0) { *ok = true; return x; }
        if (r < 0.0) lo = x; else hi = x;
        // the root lies below 1e-300 (near-Bernoulli shapes): 0 to double
        // precision, and the loss it scales underflows in FP32 anyway
        if (hi <= 1e-300) { *ok = true; return 0.0; }
        const double dens = exp(ld);
        const double u = r / dens;
        const double hh = (a - 1.0) / x - (b - 1.0) / (1.0 - x);
        const double t = u / (1.0 - 0.5 * fmin(1.0, u * hh));
        double xn = x - t;
        if (!(xn > lo && xn < hi)) {
            if (lo > 0.0 && hi > 4.0 * lo) xn = sqrt(lo * hi);
            else if (lo == 0.0) xn = 1e-3 * hi;
            else xn = 0.5 * (lo + hi);
        }
        if (fabs(xn - x) <= 1e-14 * xn || hi - lo <= 1e-15 * hi) { *ok = true; return xn; }
        x = xn;
    }
    return x;
}

// FP64 quantile (any shape a, b > 0; lnb = ln B(a, b)): the root side is
// chosen from I_{1/2}(a, b), the small side solved, the other recovered by
// 1 - y; at most max_iter steps.
__device__ inline double beta_quantile64(double a, double b, double lnb, double z, double zc,
                                        int max_iter, bool *ok) {
    double Ih, Ihc, ld;
    beta_inc64(a, b, lnb, 0.5, &Ih, &Ihc, &ld);
    const bool root_low = (z <= zc) ? (z <= Ih) : (zc >= Ihc);
    double A = a, B = b, Z = z, ZC = zc;
    if (!root_low) { A = b; B = a; Z = zc; ZC = z; }
    double x;
    if (A >= 1.0 && B >= 1.0) {
        // Abramowitz & Stegun 26.2.22 / 26.5.22 (as beta_guess32, in FP64):
        // within a few per cent of the root for shapes of any size, where the
        // small-x expansion below starts far off for large shapes
        const bool lowz = Z < 0.5;
        const double t = sqrt(-2.0 * log(lowz ? Z : ZC));
        double y = t - (2.30753 + 0.27061 * t) / (1.0 + t * (0.99229 + 0.04481 * t));
        if (!lowz) y = -y;
        const double lam = (y * y - 3.0) / 6.0;
        const double ra = 1.0 / (2.0 * A - 1.0), rb = 1.0 / (2.0 * B - 1.0);
        const double rh = 0.5 * (ra + rb);
        const double w = y * sqrt(1.0 / rh + lam) * rh - (rb - ra) * (lam + 5.0 / 6.0 - (2.0 / 3.0) * rh);
        x = A / (A + B * exp(2.0 * w));
    } else {
        // the leading term of the small-x expansion I_x ~ x^A / (A B(A, B))
        x = exp((log(Z) + log(A) + lnb) / A);
    }
    if (!(x < 0.5)) x = 0.25;
    double y = beta_solve64(A, B, lnb, Z, ZC, x, 0.5, max_iter, ok);
    if (y == 0.0) *ok = true;    // root below the smallest double
    return root_low ? y : 1.0 - y;
}

// One point of a shape table (see kShapeSlots): the logit of
// I^-1(z; a, b) at point k of half `upper` (z = p, or z = 1 - p with the
// complement p exact), solved in FP64 on both sides of the root so the
// logit keeps its precision in both tails.
__device__ inline float shape_table_logit(double a, double b, double lnb, int upper, int k) {
    const double t = kShapeTLo + (kShapeTHi - kShapeTLo) * (double)k / (double)(kShapeK - 1);
    const double p = exp(-0.5 * t * t);
    const double z = upper ? 1.0 - p : p, zc = upper ? p : 1.0 - p;
    bool ok1, ok2;
    const double x = beta_quantile64(a, b, lnb, z, zc, kF64QuantileIters, &ok1);
    const double y = beta_quantile64(b, a, lnb, zc, z, kF64QuantileIters, &ok2);   // 1 - x
    const double L = x <= 0.5 ? log(x) - log1p(-x) : log1p(-y) - log(y);
    return (float)L;
}

}  // namespace ara
