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
    uint32_t k0[10], k1[10];
};

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

inline PhiloxKeys philox_keys(uint64_t seed) {
    PhiloxKeys k;
    uint32_t a = (uint32_t)seed, b = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        k.k0[r] = a;
        k.k1[r] = b;
        a += kPhiloxW0;
        b += kPhiloxW1;
    }
    return k;
}

__device__ __forceinline__ uint4 philox10(uint4 c, const PhiloxKeys &k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)c.x;
        uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)c.z;
        uint4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k.k0[r];
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k.k1[r];
        n.w = (uint32_t)p0;
        c = n;
    }
    return c;
}

// Word 0 only: the last round's x output needs only the product M1 * c.z.
__device__ __forceinline__ uint32_t philox10_x0(uint4 c, const PhiloxKeys &k) {
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)c.x;
        uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)c.z;
        uint4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k.k0[r];
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k.k1[r];
        n.w = (uint32_t)p0;
        c = n;
    }
    return __umulhi(kPhiloxM1, c.z) ^ c.y ^ k.k0[9];
}

// Odd multiple of 2^-24: u = ((w >> 8) | 1) * 2^-24, so 1 - u is exact too.
// Returns the 24-bit odd integer j; u = j * 2^-24.
__device__ __forceinline__ uint32_t u24(uint32_t w) { return (w >> 8) | 1u; }

// ---------------------------------------------------------------------------
// FP32 building blocks
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }

// log2(1 + v) for v > -1, the rounding of w = 1 + v corrected by v / (w - 1)
// (the classical log1p construction); hardware log2 elsewhere.
__device__ __forceinline__ float log2_1p(float v) {
    float w = 1.0f + v;
    float d = w - 1.0f;
    float l = __log2f(w);
    return d == 0.0f ? v * 1.4426950408889634f : l * (v / d);
}

// Continued fraction of DLMF 8.17.22: I_x(a, b) = x^a (1-x)^b / (a B(a,b)) / K
// with K = 1 + d1/(1 + d2/(1 + ...)),
//   d_{2m+1} = -(a+m)(a+b+m) x / ((a+2m)(a+2m+1)),
//   d_{2m}   =  m(b-m) x / ((a+2m-1)(a+2m)).
// Evaluated backward from term n (more accurate in FP32 than the forward
// recurrence) without divisions: with d_j = p_j / q_j and K_j = N_j / D_j,
// N_j = q_j N_{j+1} + p_j D_{j+1}, D_j = q_j N_{j+1}; rescaled every four
// terms.  n comes from the row (enough terms at the slowest point of the
// branch, see cf_terms); lanes with fewer terms join the loop late.
// Returns 1/K.
__device__ __forceinline__ float beta_cf32(float a, float b, float x, int n, int nmax) {
    float N = 1.0f, D = 1.0f;
    const float apb = a + b;
    for (int j = nmax; j >= 1; --j) {
        const int m = j >> 1;
        const float fm = (float)m;
        float t, p;
        if (j & 1) {
            t = a + 2.0f * fm;
            p = -(a + fm) * (apb + fm) * x;
        } else {
            t = a + (2.0f * fm - 1.0f);
            p = fm * (b - fm) * x;
        }
        const float q = t * (t + 1.0f);
        if (j <= n) {
            const float Nn = q * N + p * D;
            D = q * N;
            N = Nn;
        }
        if ((j & 3) == 0) {
            const float s = rcp_f(N);
            N *= s;
            D *= s;
        }
    }
    return D / N;
}

// Terms of the continued fraction that FP32 needs (truncation below 1e-8
// relative) at the slowest point of its branch, x = (a+1)/(a+b+2); it
// converges faster for smaller x.  Evaluated in FP64 at load time; 0 when
// more than 62 terms would be needed.
__device__ inline int cf_terms(double a, double b) {
    const double x = (a + 1.0) / (a + b + 2.0);
    auto eval = [&](int n) {
        double K = 1.0;
        for (int j = n; j >= 1; --j) {
            const int m = j >> 1;
            const double d = (j & 1) ? -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0))
                                     : m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
            K = 1.0 + d / K;
        }
        return 1.0 / K;
    };
    const double ref = eval(400);
    for (int n = 2; n <= 62; n += 2)
        if (fabs(eval(n) / ref - 1.0) < 1e-8) return n;
    return 0;
}

// Initial guess: Abramowitz & Stegun 26.2.22 for the upper-tail normal
// deviate y of the smaller tail probability, then A&S 26.5.22 for the Beta
// quantile (valid for a, b > 1/2; used here for a, b >= 1).
__device__ __forceinline__ float beta_guess32(float a, float b, float z, float zc) {
    const bool lowz = z < 0.5f;
    const float pp = lowz ? z : zc;
    const float t = sqrtf(-2.0f * __logf(pp));
    float y = t - (2.30753f + 0.27061f * t) / (1.0f + t * (0.99229f + 0.04481f * t));
    if (!lowz) y = -y;                       // y = Phi^-1(1 - z)
    const float lam = (y * y - 3.0f) / 6.0f;
    const float ra = 1.0f / (2.0f * a - 1.0f), rb = 1.0f / (2.0f * b - 1.0f);
    const float h = 2.0f / (ra + rb);
    const float w = y * sqrtf(h + lam) / h - (rb - ra) * (lam + 5.0f / 6.0f - 2.0f / (3.0f * h));
    return a / (a + b * __expf(2.0f * w));
}

// I_x(a,b) (*I) and 1 - I_x(a,b) (*Ic), each on the side where it is
// accurate, and the Beta density at x; lnb2 = log2 B(a, b); na / nb the
// continued-fraction terms of the (a, b) and (b, a) branches.
__device__ __forceinline__ void beta_inc32(float a, float b, float lnb2, int na, int nb, float x,
                                           float *I, float *Ic, float *dens) {
    const float w = 1.0f - x;
    const float e2 = a * __log2f(x) + (b * log2_1p(-x) - lnb2);
    const float front = exp2f(e2);           // x^a (1-x)^b / B(a,b)
    *dens = front / (x * w);
    const bool direct = x * (a + b + 2.0f) < a + 1.0f;
    // both branches in one loop: (a, b, x) directly, else (b, a, 1 - x)
    const float A = direct ? a : b, B = direct ? b : a, X = direct ? x : w;
    const int n = direct ? na : nb;
    int nmax = n;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) nmax = max(nmax, __shfl_xor(nmax, d, 64));
    const float v = front * beta_cf32(A, B, X, n, nmax) / A;
    *I = direct ? v : 1.0f - v;
    *Ic = direct ? 1.0f - v : v;
}

// FP32 quantile x = I^-1(z; a, b) given z and zc = 1 - z (both exact), for
// shapes inside the FP32 domain (kF32MinShape <= a, b <= kF32MaxShape).
// Halley iterations on the side where the root is at most ~1/2 (mirroring
// through I_{1-x}(b,a) = 1 - z otherwise), with the residual taken on the
// side of the smaller of z, zc so it never cancels.  Returns false in *ok if
// it did not converge (the caller then uses the FP64 path).
__device__ __forceinline__ float beta_quantile32(float a, float b, float lnb2, int na, int nb,
                                                 float z, float zc, bool *ok) {
    float x0 = beta_guess32(a, b, z, zc);
    const bool mirror = x0 > 0.5f;
    float A = a, B = b, Z = z, ZC = zc;
    int NA = na, NB = nb;
    if (mirror) {
        A = b; B = a; Z = zc; ZC = z; NA = nb; NB = na;
        x0 = 1.0f - x0;
    }
    float x = fminf(fmaxf(x0, 1e-30f), 0.75f);
    const bool lower = Z <= 0.5f;
    bool conv = false;
    for (int it = 0; it < 6; ++it) {
        float I, Ic, dens;
        beta_inc32(A, B, lnb2, NA, NB, x, &I, &Ic, &dens);
        const float r = lower ? (I - Z) : (ZC - Ic);
        const float u = r / dens;
        const float hh = (A - 1.0f) * rcp_f(x) - (B - 1.0f) * rcp_f(1.0f - x);
        const float t = u / (1.0f - 0.5f * fminf(1.0f, u * hh));
        float xn = x - t;
        if (!(xn > 0.0f)) xn = 0.5f * x;
        if (!(xn < 1.0f)) xn = 0.5f * (x + 1.0f);
        conv = fabsf(xn - x) <= 6.1e-5f * xn;   // Halley: the next error ~ step^3
        x = xn;
        if (__all(conv)) break;
    }
    *ok = conv && isfinite(x);
    return mirror ? 1.0f - x : x;
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
                                      double x, double hi0, bool *ok) {
    const bool lower = z <= zc;
    double lo = 0.0, hi = hi0;
    if (!(x > 0.0 && x < hi)) x = 0.5 * hi;
    *ok = false;
    for (int it = 0; it < 400; ++it) {
        double I, Ic, ld;
        beta_inc64(a, b, lnb, x, &I, &Ic, &ld);
        const double r = lower ? (I - z) : (zc - Ic);
        if (r == 0.0) { *ok = true; return x; }
        if (r < 0.0) lo = x; else hi = x;
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
// 1 - y.
__device__ inline double beta_quantile64(double a, double b, double lnb, double z, double zc,
                                        bool *ok) {
    double Ih, Ihc, ld;
    beta_inc64(a, b, lnb, 0.5, &Ih, &Ihc, &ld);
    const bool root_low = (z <= zc) ? (z <= Ih) : (zc >= Ihc);
    double A = a, B = b, Z = z, ZC = zc;
    if (!root_low) { A = b; B = a; Z = zc; ZC = z; }
    // initial guess: the leading term of the small-x expansion
    // I_x ~ x^A / (A B(A, B)), capped inside the bracket
    double x = exp((log(Z) + log(A) + lnb) / A);
    if (!(x < 0.5)) x = 0.25;
    double y = beta_solve64(A, B, lnb, Z, ZC, x, 0.5, ok);
    if (y == 0.0) *ok = true;    // root below the smallest double
    return root_low ? y : 1.0 - y;
}

}  // namespace ara

