// Device-side building blocks of the LGF solve: complex type, compile-time roots of
// unity and register-resident pencil transforms (zero-padded forward, truncated inverse).
//
// The fast block convolution of Sec. 2.2 (Pad -> FFT -> Prod -> IFFT -> Trunc) is done
// per block/interval as three 1D passes over a [z][ky][kx] staging tile in LDS; each
// thread owns whole pencils in registers, so a pass is a register transform plus one
// LDS read and one LDS (or HBM) write per element.
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lgf_host.h"

namespace lgfdev {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T x, y;
};

// ---------------------------------------------------------------- spectrum layout
// Every spectrum array (sources, fields, kernels) is stored frequency-chunk major:
// coefficient w of item i lives at ((w / 64) * nitems + i) * 64 + w % 64.  The Prod kernels
// work one frequency chunk at a time across all items, so the data they touch together is
// contiguous (no aliasing of many items onto the same memory channels), and a wave's 64
// lanes of one item read or write one 64-coefficient run.  S is padded to a multiple of 64.
__host__ __device__ __forceinline__ int64_t spec_at(int64_t item, int w, int64_t nitems) {
    return ((int64_t)(w >> 6) * nitems + item) * kSpecChunk + (w & 63);
}

// ---------------------------------------------------------------- symmetry-reduced kernel spectra
// The LGF is invariant under the 48 signed permutations g of the axes (Sec. 2.1), and the
// kernel tiles are embedded centred (offset r at circulant index r mod M, zero at |r| = M/2),
// so the spectrum of offset g D is that of D read at the frequency g^-1 omega (Sec. 3.1,
// pre-computation, on the unique kernel vectors).  A reduced table keeps one spectrum per
// class D_c = (a, b, c), a >= b >= c >= 0; offset D = (D_0, D_1, D_2) is described by
//   info = cls | (i_0 | s_0 << 2 | i_1 << 3 | s_1 << 5 | i_2 << 6 | s_2 << 8) << 16,
// where |D_{i_0}| >= |D_{i_1}| >= |D_{i_2}| and s_j = 1 when D_{i_j} < 0: then
// nu_j = (s_j ? -1 : 1) * omega_{i_j} (mod M).  Frequencies with nu_x > M/2 lie outside the
// stored half spectrum [kz][ky][kx <= M/2] and are read as the conjugate at -nu (real
// kernels), so a reflection costs an index change, not a twiddle multiplication.
// sym: reduced-table view (info == nullptr: the table holds one spectrum per offset).
struct SpecSym {
    const uint32_t* info = nullptr;  // per offset, as above
    int ncls = 0;                    // spectra in the reduced table
    int M = 0;                       // padded tile edge
};
// Frequency (kx, ky, kz) of spectrum index w = (kz M + ky) H + kx, H = M/2 + 1.
struct Freq3 {
    int v[3];
};
__device__ __forceinline__ Freq3 freq_of(int w, int M) {
    const int H = M / 2 + 1;
    const int t = w / H;
    return Freq3{{w - t * H, t % M, t / M}};
}
template <typename T>
__device__ __forceinline__ cplx<T> sym_coef(const cplx<T>* __restrict__ khat, uint32_t info, const Freq3& om,
                                            int ncls, int M) {
    int nu[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t a = (info >> (16 + 3 * j)) & 3u;
        const int v = a == 0 ? om.v[0] : (a == 1 ? om.v[1] : om.v[2]);
        nu[j] = ((info >> (18 + 3 * j)) & 1u) && v ? M - v : v;
    }
    const bool cj = 2 * nu[0] > M;
    if (cj) {
#pragma unroll
        for (int j = 0; j < 3; ++j) nu[j] = nu[j] ? M - nu[j] : 0;
    }
    const int idx = (nu[2] * M + nu[1]) * (M / 2 + 1) + nu[0];
    cplx<T> k = khat[spec_at((int)(info & 0xffffu), idx, ncls)];
    if (cj) k.y = -k.y;
    return k;
}

// ---------------------------------------------------------------- float-float numbers
// An unevaluated sum hi + lo of two floats (|lo| <= ulp(hi)/2), with error-free
// transformations (Knuth TwoSum, FMA-based TwoProduct).  Used by the FP32 path to carry
// the far-field level contributions with compensation through the interpolation down the
// tree, where the Lebesgue constant of equispaced interpolation would otherwise amplify
// FP32 rounding of the node values.
// Every function here turns floating-point contraction off: HIP device code contracts
// a * b + c into one FMA by default, and fusing the rounded product p = a.hi * b.hi into
// the following sum p + e would break the error-free transformations (the error term is
// computed from the rounded p), leaving products with FP32 accuracy only.
struct alignas(8) ff32 {
    float hi, lo;
    ff32() = default;
    __host__ __device__ constexpr ff32(float h, float l) : hi(h), lo(l) {}
    __host__ __device__ ff32(int v) : hi((float)v), lo(0.f) {}
    __host__ __device__ ff32(float v) : hi(v), lo(0.f) {}
    __host__ __device__ ff32(double d) : hi((float)d), lo((float)(d - (double)(float)d)) {}
};

__device__ __forceinline__ ff32 ff_two_sum(float a, float b) {
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return ff32(s, e);
}
__device__ __forceinline__ ff32 ff_fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
    const float s = a + b;
    return ff32(s, b - (s - a));
}
__device__ __forceinline__ ff32 operator+(ff32 a, ff32 b) {
#pragma clang fp contract(off)
    ff32 s = ff_two_sum(a.hi, b.hi);
    s.lo += a.lo + b.lo;
    return ff_fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ ff32 operator-(ff32 a) { return ff32(-a.hi, -a.lo); }
__device__ __forceinline__ ff32 operator-(ff32 a, ff32 b) { return a + (-b); }
__device__ __forceinline__ ff32 operator*(ff32 a, ff32 b) {
#pragma clang fp contract(off)
    const float p = a.hi * b.hi;
    float e = __builtin_fmaf(a.hi, b.hi, -p);
    e = __builtin_fmaf(a.hi, b.lo, e);
    e = __builtin_fmaf(a.lo, b.hi, e);
    return ff_fast_two_sum(p, e);
}
__device__ __forceinline__ ff32& operator+=(ff32& a, ff32 b) {
    a = a + b;
    return a;
}

__device__ __forceinline__ double to_double(double v) { return v; }
__device__ __forceinline__ double to_double(float v) { return (double)v; }
__device__ __forceinline__ double to_double(ff32 v) { return (double)v.hi + (double)v.lo; }

// ---------------------------------------------------------------- compile-time roots
// cos / sin of 2*pi*k/M, reduced exactly to [0, pi/4] by integer octant arithmetic and
// then summed as Taylor series (|error| < 1e-17 on that range).
constexpr double kTwoPi = 6.283185307179586476925286766559;

constexpr double taylor_sin(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 16; ++i) {
        term *= -x2 / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double taylor_cos(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 16; ++i) {
        term *= -x2 / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}

struct Root {
    double c, s;
};

// e^{+2 pi i k / M}
constexpr Root unit_root(int k, int M) {
    k = ((k % M) + M) % M;
    // angle = (pi/2) * (4k / M) = quarter turns q plus fraction r/M of a quarter turn
    int q = (4 * k) / M;
    int r = 4 * k - q * M;  // 0 <= r < M
    double c = 1.0, s = 0.0;
    if (2 * r <= M) {
        double phi = (kTwoPi / 4.0) * r / M;
        c = taylor_cos(phi);
        s = taylor_sin(phi);
    } else {
        double phi = (kTwoPi / 4.0) * (M - r) / M;
        c = taylor_sin(phi);
        s = taylor_cos(phi);
    }
    // rotate by q quarter turns
    for (int i = 0; i < q; ++i) {
        double nc = -s, ns = c;
        c = nc;
        s = ns;
    }
    return Root{c, s};
}

template <int M>
struct RootTable {
    double c[M];
    double s[M];
    constexpr RootTable() : c(), s() {
        for (int k = 0; k < M; ++k) {
            Root r = unit_root(k, M);
            c[k] = r.c;
            s[k] = r.s;
        }
    }
};

constexpr bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
constexpr int bitrev(int i, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}

// a * w with w = (wr, wi); exact shortcuts for w in {1, -1, i, -i} once constants fold
template <typename T>
__device__ __forceinline__ void cmul_const(T ar, T ai, double wr, double wi, T& orr, T& oi) {
    if (wr == 1.0 && wi == 0.0) {
        orr = ar; oi = ai;
    } else if (wr == -1.0 && wi == 0.0) {
        orr = -ar; oi = -ai;
    } else if (wr == 0.0 && wi == 1.0) {
        orr = -ai; oi = ar;
    } else if (wr == 0.0 && wi == -1.0) {
        orr = ai; oi = -ar;
    } else if constexpr (std::is_floating_point<T>::value) {
        // fused explicitly, so the rounding does not depend on how the compiler unrolls or
        // schedules a kernel variant (every variant of a transform gives the same bits)
        const T r = (T)wr, i = (T)wi;
        orr = fma(ar, r, -(ai * i));
        oi = fma(ar, i, ai * r);
    } else {
        const T r = (T)wr, i = (T)wi;
        orr = ar * r - ai * i;
        oi = ar * i + ai * r;
    }
}

// In-place radix-2 DIT FFT of length N (power of two) in registers.
// SIGN = -1: X[k] = sum x[j] e^{-2 pi i jk/N};  SIGN = +1: unnormalised inverse.
template <typename T, int N, int SIGN>
__device__ __forceinline__ void fft_reg(T (&re)[N], T (&im)[N]) {
    constexpr int bits = ilog2(N);
    constexpr RootTable<N> R{};
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int j = bitrev(i, bits);
        if (j > i) {
            T t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
#pragma unroll
    for (int half = 1; half < N; half <<= 1) {
#pragma unroll
        for (int start = 0; start < N; start += 2 * half) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const int idx = j * (N / (2 * half));
                const double wr = R.c[idx];
                const double wi = SIGN * R.s[idx];
                const int a = start + j, b = a + half;
                T tr, ti;
                cmul_const<T>(re[b], im[b], wr, wi, tr, ti);
                re[b] = re[a] - tr;
                im[b] = im[a] - ti;
                re[a] = re[a] + tr;
                im[a] = im[a] + ti;
            }
        }
    }
}

constexpr int smallest_factor(int v) {
    for (int r = 2; r * r <= v; ++r)
        if (v % r == 0) return r;
    return v;
}

// acc + a * c for a compile-time constant c, fused where T is a machine float
template <typename T>
__device__ __forceinline__ T madd_const(T a, double c, T acc) {
    if constexpr (std::is_floating_point<T>::value)
        return fma(a, (T)c, acc);
    else
        return acc + a * T(c);
}

// In-place DFT of odd prime length N in registers, by conjugate input pairs: with
// a_j = x_j + x_{N-j} and b_j = x_j - x_{N-j} (0 < j <= h = (N - 1) / 2),
//   X_0 = x_0 + sum_j a_j,
//   X_k, X_{N-k} = x_0 + sum_j a_j cos(2 pi jk/N)  +/-  SIGN i sum_j b_j sin(2 pi jk/N),
// a quarter of the real multiplications of the direct sum.
template <typename T, int N, int SIGN>
__device__ __forceinline__ void dft_prime(T (&re)[N], T (&im)[N]) {
    constexpr int h = (N - 1) / 2;
    constexpr RootTable<N> R{};
    T ar[h + 1], ai[h + 1], br[h + 1], bi[h + 1];
    T s0r = re[0], s0i = im[0];
#pragma unroll
    for (int j = 1; j <= h; ++j) {
        ar[j] = re[j] + re[N - j];
        ai[j] = im[j] + im[N - j];
        br[j] = re[j] - re[N - j];
        bi[j] = im[j] - im[N - j];
        s0r = s0r + ar[j];
        s0i = s0i + ai[j];
    }
    T outr[N], outi[N];
    outr[0] = s0r;
    outi[0] = s0i;
#pragma unroll
    for (int k = 1; k <= h; ++k) {
        T cr = re[0], ci = im[0];
        T sr = br[1] * T(R.s[k % N]), si = bi[1] * T(R.s[k % N]);
        cr = madd_const<T>(ar[1], R.c[k % N], cr);
        ci = madd_const<T>(ai[1], R.c[k % N], ci);
#pragma unroll
        for (int j = 2; j <= h; ++j) {
            const int idx = (j * k) % N;
            cr = madd_const<T>(ar[j], R.c[idx], cr);
            ci = madd_const<T>(ai[j], R.c[idx], ci);
            sr = madd_const<T>(br[j], R.s[idx], sr);
            si = madd_const<T>(bi[j], R.s[idx], si);
        }
        // i * SIGN * (sr + i si) = SIGN * (-si + i sr)
        if constexpr (SIGN > 0) {
            outr[k] = cr - si;
            outi[k] = ci + sr;
            outr[N - k] = cr + si;
            outi[N - k] = ci - sr;
        } else {
            outr[k] = cr + si;
            outi[k] = ci - sr;
            outr[N - k] = cr - si;
            outi[N - k] = ci + sr;
        }
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        re[k] = outr[k];
        im[k] = outi[k];
    }
}

// In-place DFT of any length N in registers, X_k = sum_j x_j e^{SIGN 2 pi i jk/N}:
// radix-2 for powers of two, the conjugate-pair sum for odd primes, and otherwise one
// Cooley-Tukey step N = r N2 (r the smallest prime factor; decimation in time):
//   X_{k1 + N2 k2} = sum_{j1 < r} e^{SIGN 2 pi i j1 k2 / r} [e^{SIGN 2 pi i j1 k1 / N} Y_{j1}(k1)],
// with Y_{j1} the N2-point DFT of x_{j1}, x_{j1 + r}, x_{j1 + 2r}, ...
template <typename T, int N, int SIGN>
__device__ __forceinline__ void dft_reg(T (&re)[N], T (&im)[N]) {
    if constexpr (N == 1) {
        return;
    } else if constexpr (is_pow2(N)) {
        fft_reg<T, N, SIGN>(re, im);
    } else if constexpr (smallest_factor(N) == N) {
        dft_prime<T, N, SIGN>(re, im);
    } else {
        constexpr int r = smallest_factor(N), N2 = N / r;
        constexpr RootTable<N> R{};
        T sr[r][N2], si[r][N2];
#pragma unroll
        for (int j1 = 0; j1 < r; ++j1) {
#pragma unroll
            for (int j2 = 0; j2 < N2; ++j2) {
                sr[j1][j2] = re[j2 * r + j1];
                si[j1][j2] = im[j2 * r + j1];
            }
            dft_reg<T, N2, SIGN>(sr[j1], si[j1]);
        }
#pragma unroll
        for (int k1 = 0; k1 < N2; ++k1) {
            T tr[r], ti[r];
#pragma unroll
            for (int j1 = 0; j1 < r; ++j1) {
                const int idx = (j1 * k1) % N;
                cmul_const<T>(sr[j1][k1], si[j1][k1], R.c[idx], SIGN * R.s[idx], tr[j1], ti[j1]);
            }
            dft_reg<T, r, SIGN>(tr, ti);
#pragma unroll
            for (int k2 = 0; k2 < r; ++k2) {
                re[k1 + N2 * k2] = tr[k2];
                im[k1 + N2 * k2] = ti[k2];
            }
        }
    }
}

// Forward transform of m inputs zero-padded to M outputs:
//   X[k] = sum_{j<m} x[j] e^{-2 pi i jk/M},  k < M.
// With M = 2m: X[2k] = DFT_m(x)[k], X[2k+1] = DFT_m(x_j w^j)[k] (w = e^{-2 pi i/M}).
// Otherwise a direct DFT with compile-time roots.
template <typename T, int m, int M>
__device__ __forceinline__ void pencil_fwd(const T (&xr)[m], const T (&xi)[m], T (&Xr)[M], T (&Xi)[M]) {
    if constexpr (2 * m == M && m >= 2) {
        constexpr RootTable<M> R{};
        T er[m], ei[m], orr[m], oi[m];
#pragma unroll
        for (int j = 0; j < m; ++j) {
            er[j] = xr[j];
            ei[j] = xi[j];
            cmul_const<T>(xr[j], xi[j], R.c[j], -R.s[j], orr[j], oi[j]);
        }
        dft_reg<T, m, -1>(er, ei);
        dft_reg<T, m, -1>(orr, oi);
#pragma unroll
        for (int k = 0; k < m; ++k) {
            Xr[2 * k] = er[k];
            Xi[2 * k] = ei[k];
            Xr[2 * k + 1] = orr[k];
            Xi[2 * k + 1] = oi[k];
        }
    } else {
        constexpr RootTable<M> R{};
#pragma unroll
        for (int k = 0; k < M; ++k) {
            T sr = xr[0], si = xi[0];
#pragma unroll
            for (int j = 1; j < m; ++j) {
                const int idx = (j * k) % M;
                T tr, ti;
                cmul_const<T>(xr[j], xi[j], R.c[idx], -R.s[idx], tr, ti);
                sr += tr;
                si += ti;
            }
            Xr[k] = sr;
            Xi[k] = si;
        }
    }
}

// Truncated inverse: x[j] = sum_{k<M} X[k] e^{+2 pi i jk/M}, j < m (unnormalised).
// With M = 2m: x[j] = IDFT_m(X[2k])[j] + w^j IDFT_m(X[2k+1])[j] (w = e^{+2 pi i/M}).
template <typename T, int m, int M>
__device__ __forceinline__ void pencil_inv(const T (&Xr)[M], const T (&Xi)[M], T (&xr)[m], T (&xi)[m]) {
    if constexpr (2 * m == M && m >= 2) {
        constexpr RootTable<M> R{};
        T er[m], ei[m], orr[m], oi[m];
#pragma unroll
        for (int k = 0; k < m; ++k) {
            er[k] = Xr[2 * k];
            ei[k] = Xi[2 * k];
            orr[k] = Xr[2 * k + 1];
            oi[k] = Xi[2 * k + 1];
        }
        dft_reg<T, m, +1>(er, ei);
        dft_reg<T, m, +1>(orr, oi);
#pragma unroll
        for (int j = 0; j < m; ++j) {
            T tr, ti;
            cmul_const<T>(orr[j], oi[j], R.c[j], R.s[j], tr, ti);
            xr[j] = er[j] + tr;
            xi[j] = ei[j] + ti;
        }
    } else {
        constexpr RootTable<M> R{};
#pragma unroll
        for (int j = 0; j < m; ++j) {
            T sr = Xr[0], si = Xi[0];
#pragma unroll
            for (int k = 1; k < M; ++k) {
                const int idx = (j * k) % M;
                T tr, ti;
                cmul_const<T>(Xr[k], Xi[k], R.c[idx], R.s[idx], tr, ti);
                sr += tr;
                si += ti;
            }
            xr[j] = sr;
            xi[j] = si;
        }
    }
}

// Twiddle table for the runtime-indexed DFTs below: tw[r] = (cos, sin)(2 pi r / M), r < M,
// from the compile-time roots (staged in LDS by the caller).
template <int M>
__device__ __forceinline__ void stage_roots(double2* tw, int tid, int nthreads) {
    constexpr RootTable<M> R{};
#pragma unroll
    for (int r = 0; r < M; ++r)
        if (r % nthreads == tid) tw[r] = make_double2(R.c[r], R.s[r]);
}

// a * (wr + i wi) with runtime twiddles (exact for w in {1, -1, i, -i} as well: the FMA
// forms give a product of 0 or a copy in each term)
template <typename T>
__device__ __forceinline__ void cmul_rt(T ar, T ai, double wr, double wi, T& orr, T& oi) {
    if constexpr (std::is_floating_point<T>::value) {
        const T r = (T)wr, i = (T)wi;
        orr = fma(ar, r, -(ai * i));
        oi = fma(ar, i, ai * r);
    } else {
        const T r = (T)wr, i = (T)wi;
        orr = ar * r - ai * i;
        oi = ar * i + ai * r;
    }
}

// Direct DFT handing each output to `put` as soon as it is formed, outputs in a runtime
// loop and twiddles read from tw (large prime-factor pencils: compile-time 64-bit roots and
// all outputs live at once would spill):
//   put(k, X_k) for k < nout,  X_k = sum_{j < nin} x_j e^{SIGN 2 pi i jk / M}.
// Outputs k = k0, k0 + kstep, ... (several threads may share one pencil).
template <typename T, int nin, int M, int SIGN, int nout, typename Put>
__device__ __forceinline__ void dft_each(const T (&xr)[nin], const T (&xi)[nin], const double2* tw, Put put,
                                         int k0 = 0, int kstep = 1) {
#pragma unroll 1
    for (int k = k0; k < nout; k += kstep) {
        T sr = xr[0], si = xi[0];
        int idx = 0;
#pragma unroll
        for (int j = 1; j < nin; ++j) {
            idx += k;
            if (idx >= M) idx -= M;  // idx = j k mod M
            const double2 w = tw[idx];
            T tr, ti;
            cmul_rt<T>(xr[j], xi[j], w.x, SIGN * w.y, tr, ti);
            sr += tr;
            si += ti;
        }
        put(k, sr, si);
    }
}

// Real truncated inverse of a Hermitian spectrum from its first H = M/2 + 1 coefficients,
// one output at a time: x_j = Y_0 + (-1)^j Y_{M/2} + 2 Re sum_{0<k<M/2} Y_k e^{+2 pi i jk/M}.
template <typename T, int m, int M, typename Put>
__device__ __forceinline__ void c2r_each(const T (&Yr)[M / 2 + 1], const T (&Yi)[M / 2 + 1], const double2* tw,
                                         Put put, int j0 = 0, int jstep = 1) {
#pragma unroll 1
    for (int j = j0; j < m; j += jstep) {
        T acc = T(0);
        int idx = 0;
#pragma unroll
        for (int k = 1; k < M / 2; ++k) {
            idx += j;
            if (idx >= M) idx -= M;  // idx = j k mod M
            const double2 w = tw[idx];
            T tr, ti;
            cmul_rt<T>(Yr[k], Yi[k], w.x, w.y, tr, ti);
            acc += tr;
        }
        const T nyq = (j & 1) ? -Yr[M / 2] : Yr[M / 2];
        put(j, Yr[0] + nyq + (acc + acc));
    }
}

// Forward transform of m real inputs zero-padded to M = 2m, its first H = m + 1 outputs
// X[k] = sum_{j<m} x[j] e^{-2 pi i jk/M}, from one complex m-point DFT of the inputs packed
// two to a value, y_j = x_{2j} + i x_{2j+1}:  with Y = DFT_m(y),
//   X_k = E_k + e^{-2 pi i k/M} O_k,  E_k = (Y_k + conj Y_{m-k}) / 2,  O_k = (Y_k - conj Y_{m-k}) / 2i
// (indices of Y mod m; E and O are the m-point DFTs of the even and odd inputs).
template <typename T, int m, int M>
__device__ __forceinline__ void pencil_r2c(const T (&x)[m], T (&Xr)[M / 2 + 1], T (&Xi)[M / 2 + 1]) {
    static_assert(M == 2 * m, "padded length is twice the input length");
    constexpr RootTable<M> R{};
    T yr[m], yi[m];
#pragma unroll
    for (int j = 0; j < m; ++j) {
        yr[j] = 2 * j < m ? x[2 * j] : T(0);
        yi[j] = 2 * j + 1 < m ? x[2 * j + 1] : T(0);
    }
    dft_reg<T, m, -1>(yr, yi);
#pragma unroll
    for (int k = 0; k <= m; ++k) {
        const int a = k % m, b = (m - k) % m;
        const T er = T(0.5) * (yr[a] + yr[b]), ei = T(0.5) * (yi[a] - yi[b]);
        // O = (Y_a - conj Y_b) / 2i
        const T orr = T(0.5) * (yi[a] + yi[b]), oi = T(-0.5) * (yr[a] - yr[b]);
        T tr, ti;
        cmul_const<T>(orr, oi, R.c[k % M], -R.s[k % M], tr, ti);
        Xr[k] = er + tr;
        Xi[k] = ei + ti;
    }
}

// Real part only of the truncated inverse of a Hermitian spectrum given by its first
// H = M/2 + 1 coefficients (C2R): x[j] = sum_{k<M} Z[k] e^{+2 pi i jk/M}, Z[M-k] = conj Z[k].
// For M = 2m other than a power of two the outputs are formed two to a complex value,
// y_j = x_{2j} + i x_{2j+1} = IDFT_m(E + i O)[j], one m-point DFT, with (w = e^{+2 pi i/M})
//   E_k = Y_k + conj Y_{m-k},  O_k = (Y_k - conj Y_{m-k}) w^k   (0 < k < m),
//   E_0 = Re Y_0 + Re Y_m,     O_0 = Re Y_0 - Re Y_m,
// the even- and odd-sample spectra, Hermitian in k by construction (so both inverses are
// real).  Powers of two take the full complex pencil.
template <typename T, int m, int M>
__device__ __forceinline__ void pencil_c2r(const T (&Yr)[M / 2 + 1], const T (&Yi)[M / 2 + 1], T (&x)[m]) {
    if constexpr (!is_pow2(M) && 2 * m == M && m >= 2) {
        constexpr RootTable<M> R{};
        T cr[m], ci[m];
        cr[0] = Yr[0] + Yr[m];
        ci[0] = Yr[0] - Yr[m];
#pragma unroll
        for (int k = 1; k < m; ++k) {
            const T er = Yr[k] + Yr[m - k], ei = Yi[k] - Yi[m - k];
            const T dr = Yr[k] - Yr[m - k], di = Yi[k] + Yi[m - k];
            T orr, oi;
            cmul_const<T>(dr, di, R.c[k], R.s[k], orr, oi);
            cr[k] = er - oi;
            ci[k] = ei + orr;
        }
        dft_reg<T, m, +1>(cr, ci);
#pragma unroll
        for (int j = 0; j < m; ++j) x[j] = (j & 1) ? ci[j / 2] : cr[j / 2];
        return;
    }
    T Zr[M], Zi[M];
#pragma unroll
    for (int k = 0; k <= M / 2; ++k) {
        Zr[k] = Yr[k];
        Zi[k] = Yi[k];
    }
#pragma unroll
    for (int k = M / 2 + 1; k < M; ++k) {
        Zr[k] = Yr[M - k];
        Zi[k] = -Yi[M - k];
    }
    T xr[m], xi[m];
    pencil_inv<T, m, M>(Zr, Zi, xr, xi);
#pragma unroll
    for (int j = 0; j < m; ++j) x[j] = xr[j];
}

}  // namespace lgfdev
