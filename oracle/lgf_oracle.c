/*
 * Oracle (CPU, FP64): lattice Green's function values and brute-force direct sums.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library; the product path never links or calls it.
 *
 * 1. LGF of the 7-point Laplacian by the one-dimensional Bessel integral of
 *    Appendix A (Eq. lgf3):
 *        G(n) = - int_0^inf e^{-6t} I_{n1}(2t) I_{n2}(2t) I_{n3}(2t) dt
 *             = -1/2 int_0^inf  Ib_{n1}(x) Ib_{n2}(x) Ib_{n3}(x) dx,
 *    with Ib_k(x) = e^{-x} I_k(x) (substitution x = 2t).
 *    - Ib_0..Ib_K at one abscissa come from Miller's backward recurrence
 *      I_{k-1} = I_{k+1} + (2k/x) I_k, normalised by e^{-x}(I_0 + 2 sum_k I_k) = 1.
 *    - [0, X] is integrated in s = ln x with composite Gauss-Legendre panels (the
 *      integrand is smooth in s; Appendix A leaves the quadrature rule open).
 *    - [X, inf) is integrated term by term from the large-argument expansion of
 *      I_k (Appendix A): Ib_k(x) ~ (2 pi x)^{-1/2} sum_t (-1)^t a_t(k) x^{-t},
 *      a_t(k) = prod_{s=1..t} (4k^2 - (2s-1)^2) / (t! 8^t).
 * 2. Direct sum u(t) = sum_m G(t - m) f(m)  (Sec. 2.1, Eq. dpoissonsoln) with
 *    Neumaier-compensated accumulation, OpenMP over targets.
 * 3. The LGF of the screened operator L - kappa (a second non-oscillatory lattice kernel,
 *    Sec. 5), by the same Bessel integral with the extra factor e^{-kappa t}.
 *
 * Build:  gcc -O2 -fopenmp -shared -fPIC lgf_oracle.c -o liblgf_oracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------- Gauss-Legendre rule on [-1, 1] (Newton on P_m) ---------------- */
static void gauss_legendre(int m, double* x, double* w) {
    for (int i = 0; i < m; ++i) {
        double z = cos(M_PI * (i + 0.75) / (m + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= m; ++j) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            dp = m * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) {
                /* recompute derivative at the converged root */
                p0 = 1.0; p1 = 0.0;
                for (int j = 1; j <= m; ++j) {
                    double p2 = p1;
                    p1 = p0;
                    p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
                }
                dp = m * (z * p0 - p1) / (z * z - 1.0);
                break;
            }
        }
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ---------------- scaled modified Bessel functions by Miller recurrence ---------------- */
/* out[k] = e^{-x} I_k(x), k = 0..K. */
static void scaled_bessel_miller(double x, int K, double* out) {
    int N = K + 40 + (int)ceil(sqrt(100.0 * x));
    const double big = 1e200, small = 1e-200;
    double tk1 = 0.0;       /* t_{k+1} */
    double tk = 1e-280;     /* t_k, k = N */
    for (int k = 0; k <= K; ++k) out[k] = 0.0;
    /* Neumaier sum of t_0 + 2 sum_{k>=1} t_k, rescaled together with the t's */
    double s = 0.0, c = 0.0;
    for (int k = N; k >= 1; --k) {
        if (k <= K) out[k] = tk;
        double term = 2.0 * tk;
        double t = s + term;
        if (fabs(s) >= fabs(term)) c += (s - t) + term; else c += (term - t) + s;
        s = t;
        double tm1 = tk1 + (2.0 * k / x) * tk;  /* t_{k-1} */
        tk1 = tk;
        tk = tm1;
        if (fabs(tk) > big) {
            tk *= small; tk1 *= small; s *= small; c *= small;
            for (int j = k - 1; j <= K; ++j)
                if (j >= 0) out[j] *= small;
        }
    }
    out[0] = tk;
    {
        double term = tk;
        double t = s + term;
        if (fabs(s) >= fabs(term)) c += (s - t) + term; else c += (term - t) + s;
        s = t;
    }
    double S = s + c;
    for (int k = 0; k <= K; ++k) out[k] /= S;
}

/* coefficients a_t(k) of the large-argument expansion, t = 0..T-1 */
static void bessel_asym_coeffs(int k, int T, double* a) {
    double kk = 4.0 * k * k;
    a[0] = 1.0;
    for (int t = 1; t < T; ++t) {
        double f = (kk - (2.0 * t - 1.0) * (2.0 * t - 1.0)) / (8.0 * t);
        a[t] = a[t - 1] * f;
    }
}

/*
 * Fill G on the full octant [0,R)^3: out[(a*R + b)*R + c] = G(a, b, c).
 * Only a >= b >= c is integrated; the rest follows from the 48-fold symmetry
 * (reflections and index permutations, Sec. 2.1).
 *   xmax        : split point X of the integral
 *   panel_width : panel width in s = ln x
 *   order       : Gauss-Legendre points per panel
 * Returns 0 on success.
 */
int oracle_lgf_table(int R, double xmax, double panel_width, int order, double* out) {
    if (R < 1 || xmax <= 1.0 || panel_width <= 0.0 || order < 2) return 1;
    const double smin = log(1e-18), smax = log(xmax);
    int npan = (int)ceil((smax - smin) / panel_width);
    double h = (smax - smin) / npan;
    int nq = npan * order;
    double* gx = (double*)malloc(sizeof(double) * order);
    double* gw = (double*)malloc(sizeof(double) * order);
    gauss_legendre(order, gx, gw);
    double* xs = (double*)malloc(sizeof(double) * nq);
    double* ws = (double*)malloc(sizeof(double) * nq);
    for (int p = 0; p < npan; ++p)
        for (int i = 0; i < order; ++i) {
            double s = smin + h * (p + 0.5 * (gx[i] + 1.0));
            double x = exp(s);
            xs[p * order + i] = x;
            ws[p * order + i] = 0.5 * h * gw[i] * x; /* dx = x ds */
        }
    /* Bessel table [node][k] */
    double* Ib = (double*)malloc(sizeof(double) * (size_t)nq * R);
#pragma omp parallel for schedule(dynamic, 8)
    for (int q = 0; q < nq; ++q) scaled_bessel_miller(xs[q], R - 1, Ib + (size_t)q * R);

    /* tail coefficients */
    enum { T = 16 };
    double* ak = (double*)malloc(sizeof(double) * R * T);
    for (int k = 0; k < R; ++k) bessel_asym_coeffs(k, T, ak + k * T);

    int ntri = 0;
    for (int a = 0; a < R; ++a)
        for (int b = 0; b <= a; ++b)
            for (int c = 0; c <= b; ++c) ++ntri;
    int* tri = (int*)malloc(sizeof(int) * 3 * ntri);
    {
        int t = 0;
        for (int a = 0; a < R; ++a)
            for (int b = 0; b <= a; ++b)
                for (int c = 0; c <= b; ++c) {
                    tri[3 * t] = a; tri[3 * t + 1] = b; tri[3 * t + 2] = c; ++t;
                }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int t = 0; t < ntri; ++t) {
        int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        /* finite part, Neumaier */
        double s = 0.0, cc = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double* I = Ib + (size_t)q * R;
            double term = ws[q] * I[a] * I[b] * I[c];
            double u = s + term;
            if (fabs(s) >= fabs(term)) cc += (s - u) + term; else cc += (term - u) + s;
            s = u;
        }
        double finite = s + cc;
        /* tail: product of the three series in 1/x, then integrate x^{-3/2-m} */
        double prod[T];
        for (int m = 0; m < T; ++m) prod[m] = 0.0;
        double sa[T], sb[T], sc[T];
        for (int m = 0; m < T; ++m) {
            double sg = (m & 1) ? -1.0 : 1.0;
            sa[m] = sg * ak[a * T + m];
            sb[m] = sg * ak[b * T + m];
            sc[m] = sg * ak[c * T + m];
        }
        for (int i = 0; i < T; ++i)
            for (int j = 0; i + j < T; ++j)
                for (int k = 0; i + j + k < T; ++k) prod[i + j + k] += sa[i] * sb[j] * sc[k];
        double tail = 0.0;
        for (int m = T - 1; m >= 0; --m) tail += prod[m] * pow(xmax, -m - 0.5) / (m + 0.5);
        tail *= pow(2.0 * M_PI, -1.5);
        double g = -0.5 * (finite + tail);
        /* scatter to all permutations */
        int p[6][3] = {{a, b, c}, {a, c, b}, {b, a, c}, {b, c, a}, {c, a, b}, {c, b, a}};
        for (int k = 0; k < 6; ++k)
            out[((size_t)p[k][0] * R + p[k][1]) * R + p[k][2]] = g;
    }
    free(tri); free(ak); free(Ib); free(xs); free(ws); free(gx); free(gw);
    return 0;
}

/*
 * LGF of the screened operator L - kappa (kappa > 0; [L u](n) = sum_{+-e_i} u(n +- e_i)
 * - 6 u(n)).  Its Fourier symbol is 2cos(xi_1) + 2cos(xi_2) + 2cos(xi_3) - 6 - kappa, so the
 * derivation of Eq. lgf3 from Eq. lgf1 goes through with 6 replaced by 6 + kappa:
 *     G_kappa(n) = - int_0^inf e^{-(6 + kappa) t} I_{n1}(2t) I_{n2}(2t) I_{n3}(2t) dt
 *                = -1/2 int_0^inf e^{-kappa x / 2} Ib_{n1}(x) Ib_{n2}(x) Ib_{n3}(x) dx.
 * The factor e^{-kappa x/2} makes the integrand negligible beyond x = 80 / kappa, so the
 * integral stops at xmax with no tail term; xmax * kappa / 2 >= 40 is required.
 * out[(a*R + b)*R + c] = G_kappa(h a, h b, h c) for 0 <= a, b, c < R (lattice spacing h).
 * Returns 0 on success.
 */
int oracle_lgf_table_screened(int R, int h, double kappa, double xmax, double panel_width, int order,
                              double* out) {
    if (R < 1 || h < 1 || !(kappa > 0.0) || xmax <= 1.0 || panel_width <= 0.0 || order < 2) return 1;
    if (0.5 * kappa * xmax < 40.0) return 2;
    const double smin = log(1e-18), smax = log(xmax);
    int npan = (int)ceil((smax - smin) / panel_width);
    double hs = (smax - smin) / npan;
    int nq = npan * order;
    int K = h * (R - 1); /* highest Bessel order used */
    double* gx = (double*)malloc(sizeof(double) * order);
    double* gw = (double*)malloc(sizeof(double) * order);
    gauss_legendre(order, gx, gw);
    double* xs = (double*)malloc(sizeof(double) * nq);
    double* ws = (double*)malloc(sizeof(double) * nq);
    for (int p = 0; p < npan; ++p)
        for (int i = 0; i < order; ++i) {
            double sv = smin + hs * (p + 0.5 * (gx[i] + 1.0));
            double x = exp(sv);
            xs[p * order + i] = x;
            ws[p * order + i] = 0.5 * hs * gw[i] * x * exp(-0.5 * kappa * x); /* dx = x ds, screening */
        }
    double* Ib = (double*)malloc(sizeof(double) * (size_t)nq * (K + 1));
#pragma omp parallel for schedule(dynamic, 8)
    for (int q = 0; q < nq; ++q) scaled_bessel_miller(xs[q], K, Ib + (size_t)q * (K + 1));
    int ntri = 0;
    for (int a = 0; a < R; ++a)
        for (int b = 0; b <= a; ++b)
            for (int c = 0; c <= b; ++c) ++ntri;
    int* tri = (int*)malloc(sizeof(int) * 3 * ntri);
    {
        int t = 0;
        for (int a = 0; a < R; ++a)
            for (int b = 0; b <= a; ++b)
                for (int c = 0; c <= b; ++c) {
                    tri[3 * t] = a; tri[3 * t + 1] = b; tri[3 * t + 2] = c; ++t;
                }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int t = 0; t < ntri; ++t) {
        int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        double sm = 0.0, cc = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double* I = Ib + (size_t)q * (K + 1);
            double term = ws[q] * I[h * a] * I[h * b] * I[h * c];
            double u = sm + term;
            if (fabs(sm) >= fabs(term)) cc += (sm - u) + term; else cc += (term - u) + sm;
            sm = u;
        }
        double g = -0.5 * (sm + cc);
        int pm[6][3] = {{a, b, c}, {a, c, b}, {b, a, c}, {b, c, a}, {c, a, b}, {c, b, a}};
        for (int k = 0; k < 6; ++k)
            out[((size_t)pm[k][0] * R + pm[k][1]) * R + pm[k][2]] = g;
    }
    free(tri); free(Ib); free(xs); free(ws); free(gx); free(gw);
    return 0;
}

/* Scaled Bessel values, exported for the oracle's own self-checks. */
void oracle_scaled_bessel(double x, int K, double* out) { scaled_bessel_miller(x, K, out); }

/*
 * u[t] = sum_m G(tgt_t - src_m) f_m over all sources (Eq. dpoissonsoln).
 * G is read from a full-octant table of side R: G(d) = table[|d0|][|d1|][|d2|].
 * Returns 1 if any |d_i| >= R (nothing written then is meaningful).
 */
int oracle_direct_sum(const double* table, int R, const int32_t* src, const double* f,
                      int64_t nsrc, const int32_t* tgt, int64_t ntgt, double* u) {
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
    for (int64_t t = 0; t < ntgt; ++t) {
        int32_t tx = tgt[3 * t], ty = tgt[3 * t + 1], tz = tgt[3 * t + 2];
        double s = 0.0, c = 0.0;
        for (int64_t m = 0; m < nsrc; ++m) {
            int dx = abs(tx - src[3 * m]), dy = abs(ty - src[3 * m + 1]), dz = abs(tz - src[3 * m + 2]);
            if (dx >= R || dy >= R || dz >= R) { bad = 1; continue; }
            double term = table[((size_t)dx * R + dy) * R + dz] * f[m];
            double v = s + term;
            if (fabs(s) >= fabs(term)) c += (s - v) + term; else c += (term - v) + s;
            s = v;
        }
        u[t] = s + c;
    }
    return bad;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops above (for timing the oracle at one core and at all). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Asymptotic expansion A^q (Sec. 2.1, Eq. lgf2) at arbitrary real points.
 * Terms are T_j(x) = P_j(xhat) / (pi r^(2j+1)); P_j is given as monomials
 * xhat^e0 yhat^e1 zhat^e2 with coefficients, term j owning entries
 * [term_start[j], term_start[j+1]).  The coefficients are derived elsewhere in the
 * oracle with exact rational arithmetic.
 */
void oracle_asym_eval(const double* pts, int64_t npts, int nterms, const int32_t* term_start,
                      const int32_t* exps, const double* coefs, double* out) {
    int maxe = 0;
    for (int i = 0; i < term_start[nterms]; ++i)
        for (int d = 0; d < 3; ++d)
            if (exps[3 * i + d] > maxe) maxe = exps[3 * i + d];
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < npts; ++t) {
        double x = pts[3 * t], y = pts[3 * t + 1], z = pts[3 * t + 2];
        double r = sqrt(x * x + y * y + z * z);
        double h[3] = {x / r, y / r, z / r};
        double pw[3][64];
        for (int d = 0; d < 3; ++d) {
            pw[d][0] = 1.0;
            for (int e = 1; e <= maxe && e < 64; ++e) pw[d][e] = pw[d][e - 1] * h[d];
        }
        double acc = 0.0;
        double rpow = r; /* r^(2j+1) */
        for (int j = 0; j < nterms; ++j) {
            double v = 0.0;
            for (int i = term_start[j]; i < term_start[j + 1]; ++i)
                v += coefs[i] * pw[0][exps[3 * i]] * pw[1][exps[3 * i + 1]] * pw[2][exps[3 * i + 2]];
            acc += v / (M_PI * rpow);
            rpow *= r * r;
        }
        out[t] = acc;
    }
}
