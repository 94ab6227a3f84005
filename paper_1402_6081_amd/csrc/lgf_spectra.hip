// Step 0 of Sec. 3.1 (Eq. precomp): kernel spectra khat^{P-Q} = FFT(k^{P-Q}), generated
// on the device in FP64 and shared by every plan with the same (n, p, level, precision).
//
//  * Lattice Green's function table (Appendix A, Eq. lgf3), FP64:
//      G(n) = -1/2 int_0^inf prod_i e^{-x} I_{n_i}(x) dx.
//    One thread per quadrature abscissa runs Miller's backward recurrence for the
//    scaled Bessel functions (normalised by e^{-x}(I_0 + 2 sum I_k) = 1); one thread per
//    table entry then sums the Gauss-Legendre rule in s = ln x (compensated) and adds the
//    tail beyond X from the large-argument Bessel expansion integrated term by term.
//  * Far kernel A^q (Sec. 2.1, Eq. lgf2), q = kFarTerms: the terms are derived on the
//    host from Eq. lgf1 (expansion of 1/sigma in homogeneous parts, Fourier inversion of
//    xi^alpha |xi|^-2k as derivatives of |x|^(2k-3)) in long double.
//  * Kernel block of offset D at level l: K(D s_l + r h_l) at circular index r mod M,
//    r in [-(m-1), m-1]^3 (zero elsewhere), then three FP64 DFT passes, scaled by 1/M^3
//    so the inverse transform of a solve needs no normalisation.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>

#include "lgf_internal.h"

namespace lgfdev {

// ============================================================== quadrature (host)
namespace {

constexpr int kGLOrder = 16;
constexpr double kPanel = 0.2;
constexpr double kSLow = -46.0;      // x = e^-46 ~ 1e-20
constexpr double kXSplit = 2.0e5;    // tail starts here
constexpr int kTailTerms = 14;

void gl_rule(int m, std::vector<double>& x, std::vector<double>& w) {
    x.assign(m, 0.0);
    w.assign(m, 0.0);
    for (int i = 0; i < (m + 1) / 2; ++i) {
        long double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
        long double d = 0;
        for (int it = 0; it < 60; ++it) {
            long double a = 1, b = 0;  // P_k, P_{k-1}
            for (int k = 1; k <= m; ++k) {
                long double c = b;
                b = a;
                a = ((2 * k - 1) * z * b - (k - 1) * c) / k;
            }
            d = m * (z * a - b) / (z * z - 1);
            long double dz = a / d;
            z -= dz;
            if (std::fabs((double)dz) < 1e-19) break;
        }
        x[i] = -(double)z;
        x[m - 1 - i] = (double)z;
        w[i] = w[m - 1 - i] = (double)(2.0L / ((1 - z * z) * d * d));
    }
}

struct Quadrature {
    std::vector<double> x, w;  // abscissae in x and weights including dx = x ds
};

const Quadrature& quadrature() {
    static Quadrature q = [] {
        Quadrature Q;
        std::vector<double> gx, gw;
        gl_rule(kGLOrder, gx, gw);
        const double shi = std::log(kXSplit);
        const int npan = (int)std::ceil((shi - kSLow) / kPanel);
        const double h = (shi - kSLow) / npan;
        for (int pnl = 0; pnl < npan; ++pnl)
            for (int i = 0; i < kGLOrder; ++i) {
                const double s = kSLow + h * pnl + 0.5 * h * (gx[i] + 1.0);
                const double xv = std::exp(s);
                Q.x.push_back(xv);
                Q.w.push_back(0.5 * h * gw[i] * xv);
            }
        return Q;
    }();
    return q;
}

}  // namespace

// One thread per abscissa: scaled Bessel functions e^{-x} I_k(x), k < R, into I[q*R + k].
__global__ void k_bessel_nodes(const double* __restrict__ xs, int nq, int R, double* __restrict__ I) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const double x = xs[q];
    double* out = I + (int64_t)q * R;
    for (int k = 0; k < R; ++k) out[k] = 0.0;
    const int N = R + 40 + (int)ceil(sqrt(100.0 * x));
    double hi = 0.0, cur = 1e-290;      // t_{k+1}, t_k
    double sum = 0.0, comp = 0.0;       // Kahan sum of t_0 + 2 sum_{k>=1} t_k
    for (int k = N; k >= 1; --k) {
        if (k < R) out[k] = cur;
        {
            const double y = 2.0 * cur - comp;
            const double t = sum + y;
            comp = (t - sum) - y;
            sum = t;
        }
        const double lo = hi + (2.0 * k / x) * cur;
        hi = cur;
        cur = lo;
        if (fabs(cur) > 1e250) {
            cur *= 1e-250; hi *= 1e-250; sum *= 1e-250; comp *= 1e-250;
            for (int j = (k - 1 < 0 ? 0 : k - 1); j < R; ++j) out[j] *= 1e-250;
        }
    }
    out[0] = cur;
    {
        const double y = cur - comp;
        const double t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    }
    const double inv = 1.0 / sum;
    for (int k = 0; k < R; ++k) out[k] *= inv;
}

// LGF of the screened operator L - kappa at lattice spacing h, one thread per (a, b, c):
// the derivation of Eq. lgf3 from Eq. lgf1 holds with 6 + kappa in place of 6, i.e. the
// integrand gains the factor e^{-kappa t} = e^{-kappa x / 2}.  That factor is below e^{-40}
// beyond the last abscissa for kappa >= kKappaMin, so there is no tail term.
__global__ void k_green_table_screened(const double* __restrict__ I, const double* __restrict__ xs,
                                       const double* __restrict__ w, int nq, int K1, int R, int h, double kappa,
                                       double* __restrict__ G) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)R * R * R) return;
    const int c = (int)(id % R), b = (int)((id / R) % R), a = (int)(id / ((int64_t)R * R));
    const int ka = h * a, kb = h * b, kc = h * c;
    double sum = 0.0, comp = 0.0;
    for (int q = 0; q < nq; ++q) {
        const double* Iq = I + (int64_t)q * K1;
        const double y = w[q] * exp(-0.5 * kappa * xs[q]) * Iq[ka] * Iq[kb] * Iq[kc] - comp;
        const double t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    }
    G[id] = -0.5 * (sum - comp);
}

// One thread per (a, b, c): G[a][b][c].
__global__ void k_green_table(const double* __restrict__ I, const double* __restrict__ w, int nq, int R,
                              double xsplit, double* __restrict__ G) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)R * R * R) return;
    const int c = (int)(id % R), b = (int)((id / R) % R), a = (int)(id / ((int64_t)R * R));
    double sum = 0.0, comp = 0.0;
    for (int q = 0; q < nq; ++q) {
        const double* Iq = I + (int64_t)q * R;
        const double y = w[q] * Iq[a] * Iq[b] * Iq[c] - comp;
        const double t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    }
    // tail: prod_i sum_t (-1)^t a_t(n_i) x^-t, a_t(k) = prod_{s<=t} (4k^2 - (2s-1)^2) / (8 s)
    double sa[kTailTerms], sb[kTailTerms], sc[kTailTerms];
    const int nn[3] = {a, b, c};
    double* ser[3] = {sa, sb, sc};
    for (int d = 0; d < 3; ++d) {
        const double k4 = 4.0 * nn[d] * nn[d];
        double v = 1.0;
        ser[d][0] = 1.0;
        for (int t = 1; t < kTailTerms; ++t) {
            v *= -(k4 - (2.0 * t - 1.0) * (2.0 * t - 1.0)) / (8.0 * t);
            ser[d][t] = v;
        }
    }
    double tail = 0.0;
    for (int mdeg = kTailTerms - 1; mdeg >= 0; --mdeg) {
        double bm = 0.0;
        for (int i = 0; i <= mdeg; ++i)
            for (int j = 0; i + j <= mdeg; ++j) bm += sa[i] * sb[j] * sc[mdeg - i - j];
        tail += bm * pow(xsplit, -mdeg - 0.5) / (mdeg + 0.5);
    }
    tail *= pow(2.0 * M_PI, -1.5);
    G[id] = -0.5 * ((sum - comp) + tail);
}

// ============================================================== asymptotic expansion (host)
namespace {

using Mono = std::array<int, 3>;
using Poly = std::map<Mono, long double>;

void poly_add(Poly& a, const Poly& b, long double s) {
    for (const auto& kv : b) a[kv.first] += s * kv.second;
}
Poly poly_mul(const Poly& a, const Poly& b, int maxdeg) {
    Poly out;
    for (const auto& x : a)
        for (const auto& y : b) {
            Mono e{x.first[0] + y.first[0], x.first[1] + y.first[1], x.first[2] + y.first[2]};
            if (e[0] + e[1] + e[2] > maxdeg) continue;
            out[e] += x.second * y.second;
        }
    return out;
}
const Poly& r_squared() {
    static Poly r2{{Mono{2, 0, 0}, 1.0L}, {Mono{0, 2, 0}, 1.0L}, {Mono{0, 0, 2}, 1.0L}};
    return r2;
}
// d/dx_axis of Q r^e  ->  (dQ r^2 + e x_axis Q) r^(e-2)
Poly deriv(const Poly& Q, int e, int axis) {
    Poly dQ;
    for (const auto& kv : Q)
        if (kv.first[axis] > 0) {
            Mono m = kv.first;
            m[axis] -= 1;
            dQ[m] += kv.second * kv.first[axis];
        }
    Poly out = poly_mul(dQ, r_squared(), 1 << 20);
    for (const auto& kv : Q) {
        Mono m = kv.first;
        m[axis] += 1;
        out[m] += (long double)e * kv.second;
    }
    return out;
}
// d^alpha r^e, applying z then y then x derivatives
Poly deriv_power(const Mono& alpha, int e) {
    static std::map<std::pair<Mono, int>, Poly> memo;
    auto key = std::make_pair(alpha, e);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    Poly res;
    if (alpha[0] == 0 && alpha[1] == 0 && alpha[2] == 0) {
        res[Mono{0, 0, 0}] = 1.0L;
    } else {
        int axis = alpha[2] > 0 ? 2 : (alpha[1] > 0 ? 1 : 0);
        Mono prev = alpha;
        prev[axis] -= 1;
        const int order = prev[0] + prev[1] + prev[2];
        res = deriv(deriv_power(prev, e), e - 2 * order, axis);
    }
    memo[key] = res;
    return res;
}

// P_j with T_j(x) = P_j(x) / (pi r^(6j+1)); degree 4j
Poly asymptotic_term(int j) {
    // delta(xi) = sum_i sum_{k>=2} 2(-1)^k xi_i^(2k)/(2k)!, up to degree 2j+4
    Poly delta;
    long double fact = 2.0L;  // (2k)! for k = 1
    for (int k = 2; 2 * k <= 2 * j + 4; ++k) {
        fact *= (2.0L * k - 1) * (2.0L * k);
        const long double cf = 2.0L * ((k % 2) ? -1.0L : 1.0L) / fact;
        for (int a = 0; a < 3; ++a) {
            Mono m{0, 0, 0};
            m[a] = 2 * k;
            delta[m] += cf;
        }
    }
    Poly total;
    Poly dm{{Mono{0, 0, 0}, 1.0L}};
    long double gamma = 0.25L;  // gamma_1; F_k = gamma_k / pi * r^(2k-3)
    for (int m = 0; m <= j; ++m) {
        if (m > 0) {
            dm = poly_mul(dm, delta, 2 * j + 2 * m);
            gamma = -gamma / ((2.0L * (m + 1) - 3) * (2.0L * (m + 1) - 2));
        }
        Poly part;
        for (const auto& kv : dm) {
            const int deg = kv.first[0] + kv.first[1] + kv.first[2];
            if (deg != 2 * m + 2 * j) continue;
            const long double sign = ((deg / 2) % 2) ? -1.0L : 1.0L;
            poly_add(part, deriv_power(kv.first, 2 * m - 1), sign * kv.second);
        }
        for (int t = 0; t < j - m; ++t) part = poly_mul(part, r_squared(), 1 << 20);
        poly_add(total, part, -gamma);
    }
    Poly clean;
    for (const auto& kv : total)
        if (kv.second != 0.0L) clean[kv.first] = kv.second;
    return clean;
}

struct AsymTable {
    std::vector<int32_t> start;  // q + 1
    std::vector<int32_t> exps;   // 3 per monomial
    std::vector<double> coef;
    int maxdeg = 0;
};

const AsymTable& asym_table() {
    static AsymTable t = [] {
        AsymTable T;
        T.start.push_back(0);
        for (int j = 0; j < kFarTerms; ++j) {
            for (const auto& kv : asymptotic_term(j)) {
                for (int d = 0; d < 3; ++d) T.exps.push_back(kv.first[d]);
                T.coef.push_back((double)kv.second);
                T.maxdeg = std::max(T.maxdeg, std::max(kv.first[0], std::max(kv.first[1], kv.first[2])));
            }
            T.start.push_back((int32_t)T.coef.size());
        }
        return T;
    }();
    return t;
}

}  // namespace

struct AsymDev {
    const int32_t* start;
    const int32_t* exps;
    const double* coef;
    int nterms;
};

__device__ double eval_asym(const AsymDev& A, double x, double y, double z) {
    const double r2 = x * x + y * y + z * z;
    const double r = sqrt(r2);
    const double h[3] = {x / r, y / r, z / r};
    double pw[3][32];
    for (int d = 0; d < 3; ++d) {
        pw[d][0] = 1.0;
        for (int e = 1; e < 32; ++e) pw[d][e] = pw[d][e - 1] * h[d];
    }
    double acc = 0.0, rp = r;
    for (int j = 0; j < A.nterms; ++j) {
        double v = 0.0;
        for (int i = A.start[j]; i < A.start[j + 1]; ++i)
            v += A.coef[i] * pw[0][A.exps[3 * i]] * pw[1][A.exps[3 * i + 1]] * pw[2][A.exps[3 * i + 2]];
        acc += v / (M_PI * rp);
        rp *= r2;
    }
    return acc;
}

__global__ void k_far_kernel(const double* __restrict__ pts, int64_t npts, AsymDev A, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npts) return;
    out[i] = eval_asym(A, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
}

// kernel block, one real M^3 array per offset (blockIdx.y = offset id)
//   mode 0: exact G (table) at integer points
//   mode 1: lattice nodes: G where max|x_i| < kLatticeRadius, A^q elsewhere
//   mode 2: A^q everywhere
//   mode 3: the screened LGF from a table at lattice spacing hg (every point is a multiple)
__global__ void k_kernel_block(double* __restrict__ out, int M, int m, int radius, double s, double h, int mode,
                               const double* __restrict__ G, int Rg, AsymDev A, int hg) {
    const int M3 = M * M * M;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M3) return;
    const int o = blockIdx.y;
    const int W = 2 * radius + 1;
    const int D[3] = {o % W - radius, (o / W) % W - radius, o / (W * W) - radius};
    const int ii[3] = {idx % M, (idx / M) % M, idx / (M * M)};  // x, y, z
    int r[3];
    bool valid = true;
    for (int d = 0; d < 3; ++d) {
        if (ii[d] < m) r[d] = ii[d];
        else if (ii[d] > M - m) r[d] = ii[d] - M;
        else { valid = false; r[d] = 0; }
    }
    double v = 0.0;
    if (valid) {
        if (mode == 3) {
            const double x = D[0] * s + r[0] * h, y = D[1] * s + r[1] * h, z = D[2] * s + r[2] * h;
            const int a0 = (int)rint(fabs(x)) / hg, a1 = (int)rint(fabs(y)) / hg, a2 = (int)rint(fabs(z)) / hg;
            v = G[((int64_t)a0 * Rg + a1) * Rg + a2];
        } else if (mode == 0) {
            const int a0 = abs(D[0] * (int)s + r[0]), a1 = abs(D[1] * (int)s + r[1]), a2 = abs(D[2] * (int)s + r[2]);
            v = G[((int64_t)a0 * Rg + a1) * Rg + a2];
        } else {
            const double x = D[0] * s + r[0] * h, y = D[1] * s + r[1] * h, z = D[2] * s + r[2] * h;
            bool use_table = false;
            int a0 = 0, a1 = 0, a2 = 0;
            if (mode == 1) {
                a0 = (int)fabs(rint(x)); a1 = (int)fabs(rint(y)); a2 = (int)fabs(rint(z));
                use_table = a0 < kLatticeRadius && a1 < kLatticeRadius && a2 < kLatticeRadius;
            }
            v = use_table ? G[((int64_t)a0 * Rg + a1) * Rg + a2] : eval_asym(A, x, y, z);
        }
    }
    out[(int64_t)o * M3 + idx] = v;
}

// DFT along the middle axis of data viewed as [A][len][C] (complex), forward sign,
// with a host-prepared root table tw[k] = (cos, sin)(2 pi k / len).
__global__ void k_dft_axis(const cplx<double>* __restrict__ in, cplx<double>* __restrict__ out, int64_t A, int len,
                           int64_t C, const double* __restrict__ tw) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= A * len * C) return;
    const int64_t c = id % C;
    const int k = (int)((id / C) % len);
    const int64_t a = id / (C * len);
    const cplx<double>* src = in + a * len * C + c;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < len; ++j) {
        const int t = (int)(((int64_t)j * k) % len);
        const double wr = tw[2 * t], wi = -tw[2 * t + 1];
        const cplx<double> v = src[(int64_t)j * C];
        sr += v.x * wr - v.y * wi;
        si += v.x * wi + v.y * wr;
    }
    out[id] = cplx<double>{sr, si};
}

// real-to-complex DFT along x of real [B][M][M][M] -> complex [B][M][M][M/2+1]
__global__ void k_dft_r2c_x(const double* __restrict__ in, cplx<double>* __restrict__ out, int64_t rows, int M,
                            const double* __restrict__ tw) {
    const int H = M / 2 + 1;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= rows * H) return;
    const int k = (int)(id % H);
    const int64_t row = id / H;
    const double* src = in + row * M;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < M; ++j) {
        const int t = (j * k) % M;
        sr += src[j] * tw[2 * t];
        si -= src[j] * tw[2 * t + 1];
    }
    out[id] = cplx<double>{sr, si};
}

// scale, cast and scatter rows of [*][S] into the chunk-major layout of nout items: item o
// takes row rows[o] (rows == nullptr: row o)
template <typename T>
__global__ void k_scale_cast(const cplx<double>* __restrict__ in, cplx<T>* __restrict__ out, int nout, int S,
                             double scale, const int32_t* __restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nout * S) return;
    const int o = (int)(i / S), w = (int)(i % S);
    const cplx<double> v = in[(int64_t)(rows ? rows[o] : o) * S + w];
    out[spec_at(o, w, nout)] = cplx<T>{(T)(v.x * scale), (T)(v.y * scale)};
}

// ============================================================== host glue
namespace {

std::mutex g_mu;

struct DevAsym {
    int32_t* start = nullptr;
    int32_t* exps = nullptr;
    double* coef = nullptr;
};

bool upload_asym(DevAsym& d, std::string& err) {
    if (d.coef) return true;
    const AsymTable& t = asym_table();
    if (hipMalloc(&d.start, t.start.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&d.exps, t.exps.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&d.coef, t.coef.size() * sizeof(double)) != hipSuccess) {
        err = "hipMalloc failed for the asymptotic-expansion coefficients";
        return false;
    }
    hipMemcpy(d.start, t.start.data(), t.start.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    hipMemcpy(d.exps, t.exps.data(), t.exps.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    hipMemcpy(d.coef, t.coef.data(), t.coef.size() * sizeof(double), hipMemcpyHostToDevice);
    return true;
}

std::map<int, DevAsym> g_asym;             // per device
std::map<std::pair<int, int>, double*> g_green;  // (device, R) -> table

AsymDev asym_view(int dev) {
    const DevAsym& d = g_asym[dev];
    return AsymDev{d.start, d.exps, d.coef, kFarTerms};
}

std::vector<double> root_table(int M) {
    std::vector<double> tw(2 * M);
    for (int k = 0; k < M; ++k) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * k / M;
        tw[2 * k] = (double)std::cos(a);
        tw[2 * k + 1] = (double)std::sin(a);
    }
    return tw;
}

std::map<SpectraKey, std::shared_ptr<SpectraEntry>> g_cache;

int current_device() {
    int d = 0;
    hipGetDevice(&d);
    return d;
}

}  // namespace

bool SpectraKey::operator<(const SpectraKey& o) const {
    return std::make_tuple(n, p, level, radius, prec, m, sym, kappa) <
           std::make_tuple(o.n, o.p, o.level, o.radius, o.prec, o.m, o.sym, o.kappa);
}

SpectraEntry::~SpectraEntry() {
    if (dev_info) hipFree(dev_info);
    if (dev) {
        hipFree(dev);
        budget_release(bytes);
    }
}

namespace {
std::atomic<int> g_spectra_mode{0};
thread_local int t_spectra_mode = -1;  // a thread's own mode, or -1: the process-wide one
}
void spectra_set_mode(int mode) { g_spectra_mode.store(mode ? 1 : 0); }
void spectra_set_thread_mode(int mode) { t_spectra_mode = mode < 0 ? -1 : (mode ? 1 : 0); }
int spectra_mode() { return t_spectra_mode >= 0 ? t_spectra_mode : g_spectra_mode.load(); }

int spectra_classes(int R, std::vector<uint32_t>& info, std::vector<int32_t>& rep_offset) {
    const int W = 2 * R + 1;
    auto offset = [&](int x, int y, int z) { return (x + R) + W * ((y + R) + W * (z + R)); };
    // classes a >= b >= c >= 0, numbered in this order
    std::vector<int32_t> cls_of((size_t)W * W * W, -1);
    rep_offset.clear();
    for (int a = 0; a <= R; ++a)
        for (int b = 0; b <= a; ++b)
            for (int c = 0; c <= b; ++c) {
                cls_of[offset(a, b, c)] = (int32_t)rep_offset.size();
                rep_offset.push_back(offset(a, b, c));
            }
    info.assign((size_t)W * W * W, 0u);
    for (int z = -R; z <= R; ++z)
        for (int y = -R; y <= R; ++y)
            for (int x = -R; x <= R; ++x) {
                const int D[3] = {x, y, z};
                int ax[3] = {0, 1, 2};  // axes by decreasing |D|, ties in axis order
                std::stable_sort(ax, ax + 3, [&](int u, int v) { return std::abs(D[u]) > std::abs(D[v]); });
                const uint32_t cls =
                    (uint32_t)cls_of[offset(std::abs(D[ax[0]]), std::abs(D[ax[1]]), std::abs(D[ax[2]]))];
                uint32_t g = 0;
                for (int j = 0; j < 3; ++j) g |= (uint32_t)(ax[j] | (D[ax[j]] < 0 ? 4 : 0)) << (3 * j);
                info[offset(x, y, z)] = cls | (g << 16);
            }
    return (int)rep_offset.size();
}

static const double* green_table_locked(int R, hipStream_t s, std::string& err) {
    const int dev = current_device();
    auto it = g_green.find({dev, R});
    if (it != g_green.end()) return it->second;
    const Quadrature& Q = quadrature();
    const int nq = (int)Q.x.size();
    double *dx = nullptr, *dw = nullptr, *dI = nullptr, *dG = nullptr;
    const size_t gbytes = (size_t)R * R * R * sizeof(double);
    if (hipMalloc(&dx, nq * sizeof(double)) != hipSuccess || hipMalloc(&dw, nq * sizeof(double)) != hipSuccess ||
        hipMalloc(&dI, (size_t)nq * R * sizeof(double)) != hipSuccess || hipMalloc(&dG, gbytes) != hipSuccess) {
        err = "hipMalloc failed for the Green's function table";
        if (dx) hipFree(dx);
        if (dw) hipFree(dw);
        if (dI) hipFree(dI);
        if (dG) hipFree(dG);
        return nullptr;
    }
    hipMemcpyAsync(dx, Q.x.data(), nq * sizeof(double), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dw, Q.w.data(), nq * sizeof(double), hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_bessel_nodes, dim3((nq + 63) / 64), dim3(64), 0, s, dx, nq, R, dI);
    const int64_t tot = (int64_t)R * R * R;
    hipLaunchKernelGGL(k_green_table, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, dI, dw, nq, R, kXSplit, dG);
    hipError_t e = hipStreamSynchronize(s);
    hipFree(dx);
    hipFree(dw);
    hipFree(dI);
    if (e != hipSuccess) {
        err = std::string("Green's function table kernels failed: ") + hipGetErrorString(e);
        hipFree(dG);
        return nullptr;
    }
    g_green[{dev, R}] = dG;
    return dG;
}

const double* green_table_device(int R, hipStream_t s, std::string& err) {
    std::lock_guard<std::mutex> lk(g_mu);
    return green_table_locked(R, s, err);
}

namespace {
std::map<std::tuple<int, int, int, double>, double*> g_screened;  // (device, R, h, kappa) -> table
}

static const double* screened_table_locked(int R, int h, double kappa, hipStream_t s, std::string& err) {
    const int dev = current_device();
    const auto key = std::make_tuple(dev, R, h, kappa);
    auto it = g_screened.find(key);
    if (it != g_screened.end()) return it->second;
    if (!(kappa >= kKappaMin) || R < 1 || h < 1) {
        err = "screened LGF table: bad arguments";
        return nullptr;
    }
    const Quadrature& Q = quadrature();
    const int nq = (int)Q.x.size();
    const int K1 = h * (R - 1) + 1;  // Bessel orders 0 .. h (R - 1)
    double *dx = nullptr, *dw = nullptr, *dI = nullptr, *dG = nullptr;
    const size_t gbytes = (size_t)R * R * R * sizeof(double);
    if (hipMalloc(&dx, nq * sizeof(double)) != hipSuccess || hipMalloc(&dw, nq * sizeof(double)) != hipSuccess ||
        hipMalloc(&dI, (size_t)nq * K1 * sizeof(double)) != hipSuccess || hipMalloc(&dG, gbytes) != hipSuccess) {
        err = "hipMalloc failed for the screened Green's function table";
        if (dx) hipFree(dx);
        if (dw) hipFree(dw);
        if (dI) hipFree(dI);
        if (dG) hipFree(dG);
        return nullptr;
    }
    hipMemcpyAsync(dx, Q.x.data(), nq * sizeof(double), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dw, Q.w.data(), nq * sizeof(double), hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_bessel_nodes, dim3((nq + 63) / 64), dim3(64), 0, s, dx, nq, K1, dI);
    const int64_t tot = (int64_t)R * R * R;
    hipLaunchKernelGGL(k_green_table_screened, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, dI, dx, dw, nq,
                       K1, R, h, kappa, dG);
    hipError_t e = hipStreamSynchronize(s);
    hipFree(dx);
    hipFree(dw);
    hipFree(dI);
    if (e != hipSuccess) {
        err = std::string("screened Green's function table kernels failed: ") + hipGetErrorString(e);
        hipFree(dG);
        return nullptr;
    }
    g_screened[key] = dG;
    return dG;
}

const double* screened_table_device(int R, int h, double kappa, hipStream_t s, std::string& err) {
    std::lock_guard<std::mutex> lk(g_mu);
    return screened_table_locked(R, h, kappa, s, err);
}

hipError_t far_kernel_device(const double* pts, int64_t npts, double* out, hipStream_t s, std::string& err) {
    std::lock_guard<std::mutex> lk(g_mu);
    const int dev = current_device();
    if (!upload_asym(g_asym[dev], err)) return hipErrorOutOfMemory;
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_far_kernel, dim3((unsigned)((npts + 127) / 128)), dim3(128), 0, s, pts, npts,
                       asym_view(dev), out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free far kernel
// For callers that cannot allocate device memory (work under graph capture, serving loops,
// harnesses that forbid it): the points, the values and the expansion's coefficient tables
// are staged in one file-scope device array instead of buffers allocated per call.  Every GPU
// holds its own copy of the array for the life of the process; its device address is looked
// up once per device, and that address, never the array's name, is what host code passes to
// copies and kernels.  Calls are serialised by a lock, since they all use the one array.
constexpr int64_t kNoAllocTableBytes = 64 << 10;  // room for the coefficient tables
constexpr int64_t kNoAllocBytes = kNoAllocTableBytes + (int64_t)LGF_FAR_KERNEL_NOALLOC_MAX_POINTS * 32;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_noalloc_mu;
std::map<int, unsigned char*> g_noalloc_ptr;  // device -> address of its copy of the array
inline int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }
}  // namespace

hipError_t far_kernel_noalloc(const double* pts, int64_t npts, double* out, std::string& err) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    const int dev = current_device();
    auto it = g_noalloc_ptr.find(dev);
    if (it == g_noalloc_ptr.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("device address of the staging array: ") + hipGetErrorString(e);
            return e != hipSuccess ? e : hipErrorInvalidSymbol;
        }
        it = g_noalloc_ptr.emplace(dev, static_cast<unsigned char*>(p)).first;
    }
    unsigned char* base = it->second;
    const AsymTable& t = asym_table();
    const int64_t o_start = 0;
    const int64_t o_exps = align256(o_start + (int64_t)(t.start.size() * sizeof(int32_t)));
    const int64_t o_coef = align256(o_exps + (int64_t)(t.exps.size() * sizeof(int32_t)));
    const int64_t o_pts = align256(o_coef + (int64_t)(t.coef.size() * sizeof(double)));
    const int64_t o_out = o_pts + npts * 24;
    if (o_pts > kNoAllocTableBytes || o_out + npts * 8 > kNoAllocBytes) {
        err = "staging array too small";
        return hipErrorInvalidValue;
    }
    // the tables are copied on every call: the array keeps whatever the previous call left in it
    hipError_t e = hipMemcpy(base + o_start, t.start.data(), t.start.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + o_exps, t.exps.data(), t.exps.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + o_coef, t.coef.data(), t.coef.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + o_pts, pts, (size_t)npts * 24, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        err = std::string("copy to the staging array: ") + hipGetErrorString(e);
        return e;
    }
    const AsymDev A{reinterpret_cast<const int32_t*>(base + o_start), reinterpret_cast<const int32_t*>(base + o_exps),
                    reinterpret_cast<const double*>(base + o_coef), kFarTerms};
    hipLaunchKernelGGL(k_far_kernel, dim3((unsigned)((npts + 127) / 128)), dim3(128), 0, nullptr,
                       reinterpret_cast<const double*>(base + o_pts), npts, A, reinterpret_cast<double*>(base + o_out));
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) e = hipMemcpy(out, base + o_out, (size_t)npts * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) err = std::string("far kernel from the staging array: ") + hipGetErrorString(e);
    return e;
}

std::shared_ptr<SpectraEntry> get_spectra(const SpectraKey& key, hipStream_t s, std::string& err) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) return it->second;
    const int dev = current_device();
    if (!upload_asym(g_asym[dev], err)) return nullptr;

    const int m = key.m > 0 ? key.m : (key.level == 0 ? key.n : key.p);
    const int M = 2 * m;
    const int H = M / 2 + 1;
    const int S = M * M * H;
    const int W = 2 * key.radius + 1;
    const int noff = W * W * W;
    int mode = 0;
    double sl = key.n, hl = 1.0;
    if (key.level >= 1) {
        const int64_t sint = (int64_t)key.n << (key.level - 1);
        sl = (double)sint;
        hl = sl / (key.p - 1);
        mode = (sint % (key.p - 1) == 0) ? 1 : 2;
    }
    int Rg = std::max(2 * key.n, kLatticeRadius);
    int hg = 1;  // lattice spacing of the table
    const double* G = nullptr;
    if (key.kappa > 0.0) {
        // the screened kernel is integrated at every point it is used: a table at the
        // level's node spacing out to the farthest offset (every node is on the lattice)
        if (mode == 2) {
            err = "the screened operator needs nodes on the lattice";
            return nullptr;
        }
        hg = key.level == 0 ? 1 : (int)std::llround(hl);
        const int64_t reach = (int64_t)std::llround(key.radius * sl + (m - 1) * hl);
        Rg = (int)(reach / hg) + 1;
        mode = 3;
        G = screened_table_locked(Rg, hg, key.kappa, s, err);
    } else {
        G = green_table_locked(Rg, s, err);
    }
    if (!G) return nullptr;

    auto entry = std::make_shared<SpectraEntry>();
    entry->key = key;
    entry->M = M;
    entry->S = S;
    entry->noff = noff;
    const size_t esz = key.prec == 0 ? sizeof(cplx<double>) : sizeof(cplx<float>);
    // reduced table: the class representatives' rows of the full table, and each offset's
    // description
    std::vector<uint32_t> info;
    std::vector<int32_t> rep;
    const int nrows = key.sym ? spectra_classes(key.radius, info, rep) : noff;
    entry->bytes = (int64_t)nrows * spec_padded(S) * esz + (int64_t)info.size() * sizeof(uint32_t);
    if (!budget_reserve(entry->bytes)) {
        err = "kernel spectra exceed the device-memory budget";
        return nullptr;
    }
    const int64_t M3 = (int64_t)M * M * M;
    double* kb = nullptr;
    cplx<double> *t1 = nullptr, *t2 = nullptr;
    double* dtw = nullptr;
    int32_t* drep = nullptr;
    bool ok = hipMalloc(&entry->dev, (size_t)nrows * spec_padded(S) * esz) == hipSuccess;
    if (key.sym) {
        ok = ok && hipMalloc(&entry->dev_info, info.size() * sizeof(uint32_t)) == hipSuccess;
        ok = ok && hipMalloc(&drep, rep.size() * sizeof(int32_t)) == hipSuccess;
    }
    ok = ok && hipMalloc(&kb, noff * M3 * sizeof(double)) == hipSuccess;
    ok = ok && hipMalloc(&t1, (size_t)noff * S * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&t2, (size_t)noff * S * sizeof(cplx<double>)) == hipSuccess;
    ok = ok && hipMalloc(&dtw, 2 * M * sizeof(double)) == hipSuccess;
    if (!ok) {
        err = "hipMalloc failed while generating kernel spectra";
        if (kb) hipFree(kb);
        if (t1) hipFree(t1);
        if (t2) hipFree(t2);
        if (dtw) hipFree(dtw);
        if (drep) hipFree(drep);
        if (entry->dev_info) {
            hipFree(entry->dev_info);
            entry->dev_info = nullptr;
        }
        if (entry->dev) {
            hipFree(entry->dev);
            entry->dev = nullptr;
        }
        budget_release(entry->bytes);
        return nullptr;
    }
    if (key.sym) {
        hipMemcpyAsync(entry->dev_info, info.data(), info.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s);
        hipMemcpyAsync(drep, rep.data(), rep.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
        entry->sym = SpecSym{entry->dev_info, nrows, M};
    }
    const std::vector<double> tw = root_table(M);
    hipMemcpyAsync(dtw, tw.data(), 2 * M * sizeof(double), hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_kernel_block, dim3((unsigned)((M3 + 255) / 256), noff), dim3(256), 0, s, kb, M, m,
                       key.radius, sl, hl, mode, G, Rg, asym_view(dev), hg);
    // x: real rows -> half spectrum; then y and z complex passes
    const int64_t rows = (int64_t)noff * M * M;
    hipLaunchKernelGGL(k_dft_r2c_x, dim3((unsigned)((rows * H + 255) / 256)), dim3(256), 0, s, kb, t1, rows, M, dtw);
    const int64_t tot = (int64_t)noff * S;
    hipLaunchKernelGGL(k_dft_axis, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, t1, t2,
                       (int64_t)noff * M, M, (int64_t)H, dtw);
    hipLaunchKernelGGL(k_dft_axis, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, t2, t1, (int64_t)noff, M,
                       (int64_t)M * H, dtw);
    const double scale = 1.0 / (double)M3;
    const int64_t tout = (int64_t)nrows * S;
    if (key.prec == 0)
        hipLaunchKernelGGL(k_scale_cast<double>, dim3((unsigned)((tout + 255) / 256)), dim3(256), 0, s, t1,
                           (cplx<double>*)entry->dev, nrows, S, scale, (const int32_t*)drep);
    else
        hipLaunchKernelGGL(k_scale_cast<float>, dim3((unsigned)((tout + 255) / 256)), dim3(256), 0, s, t1,
                           (cplx<float>*)entry->dev, nrows, S, scale, (const int32_t*)drep);
    hipError_t e = hipStreamSynchronize(s);
    hipFree(kb);
    hipFree(t1);
    hipFree(t2);
    hipFree(dtw);
    if (drep) hipFree(drep);
    if (e != hipSuccess) {
        err = std::string("kernel spectra generation failed: ") + hipGetErrorString(e);
        return nullptr;
    }
    g_cache[key] = entry;
    return entry;
}

int64_t spectra_bytes_total() {
    std::lock_guard<std::mutex> lk(g_mu);
    int64_t b = 0;
    for (const auto& kv : g_cache) b += kv.second->bytes;
    return b;
}

void spectra_trim() {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
        if (it->second.use_count() == 1) it = g_cache.erase(it);
        else ++it;
    }
}

}  // namespace lgfdev
