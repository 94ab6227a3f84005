// Regularization (Reg, Eq. alg_reg / kcprss1) and interpolation (Interp, Eq. alg_interp
// / kcprss3) between levels, as tensor products of 1D Lagrange matrices (Sec. 2.5):
//   block -> level-1 interval   ftilde = (A x A x A) f           A[k][j] = phi_k(j (p-1)/n)
//   children -> parent          ftilde_J = sum_c (C_c x C_c x C_c) ftilde_{2J+c}
//                                                                 C_c[m][k] = phi_m((c(p-1)+k)/2)
//   parent -> children (add)    utilde_{2J+c} += (C_c^T x C_c^T x C_c^T) utilde_J
//   level-1 interval -> block   u = vnear + (A^T x A^T x A^T) utilde    (FP64 add-back)
// Each 3D product is three 1D passes through LDS.  Parent-level kernels handle all eight
// children of one parent per workgroup; the down pass shares the x and y passes of the
// children that have equal x (and y) child bits.
#include <type_traits>

#include "lgf_internal.h"

namespace lgfdev {

constexpr int kInterpThreads = 256;
// Reg up runs one workgroup per parent over eight children: more waves per workgroup
// hide the latency of its few, long workgroups
constexpr int kRegUpThreads = 1024;
// the per-block transfers (Reg 0->1, the final pass)
constexpr int kBlockThreads = 512;
// Interp down (one workgroup per parent, or per (parent, child))
constexpr int kDownThreads = 512;

// ------------------------------------------------------------------ block -> level 1
// One workgroup per block: the block is staged in LDS with coalesced loads, then the
// three passes run from LDS with compile-time extents.  Rows that a wave reads at several
// indices at once (the block's x rows, the matrix rows) are padded to N + 1 values, so
// the reads fall into different LDS banks.
template <typename T, int N, int P>
__global__ void __launch_bounds__(kBlockThreads)
    k_reg_block(const T* __restrict__ f, const double* __restrict__ A, T* __restrict__ out) {
    constexpr int N3 = N * N * N, P3 = P * P * P, NR = N + 1;
    __shared__ T X[N * N * NR], t1[N * N * P], t2[N * P * P];
    __shared__ T Am[P * NR];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    for (int i = tid; i < P * N; i += kBlockThreads) Am[(i / N) * NR + i % N] = (T)A[i];
    const T* src = f + b * N3;
    for (int i = tid; i < N3; i += kBlockThreads) X[(i / N) * NR + i % N] = src[i];
    __syncthreads();
    for (int i = tid; i < N * N * P; i += kBlockThreads) {  // x: t1[z][y][d]
        const int d = i % P, zy = i / P;
        const T* row = X + zy * NR;
        const T* m = Am + d * NR;
        T acc = T(0);
#pragma unroll
        for (int x = 0; x < N; ++x) acc += m[x] * row[x];
        t1[i] = acc;
    }
    __syncthreads();
    for (int i = tid; i < N * P * P; i += kBlockThreads) {  // y: t2[z][c][d]
        const int d = i % P, c = (i / P) % P, z = i / (P * P);
        const T* m = Am + c * NR;
        const T* col = t1 + z * N * P + d;
        T acc = T(0);
#pragma unroll
        for (int y = 0; y < N; ++y) acc += m[y] * col[y * P];
        t2[i] = acc;
    }
    __syncthreads();
    T* o = out + b * P3;
    for (int i = tid; i < P3; i += kBlockThreads) {  // z: out[a][c][d]
        const int cd = i % (P * P), a = i / (P * P);
        const T* m = Am + a * NR;
        T acc = T(0);
#pragma unroll
        for (int z = 0; z < N; ++z) acc += m[z] * t2[z * (P * P) + cd];
        o[i] = acc;
    }
}

// ------------------------------------------------------------------ children -> parent
template <typename T, int P, int NT = kRegUpThreads>
__global__ void __launch_bounds__(NT)
    k_reg_up(const T* __restrict__ in, const int32_t* __restrict__ child8, const double* __restrict__ C01,
             T* __restrict__ out) {
    constexpr int P3 = P * P * P;
    __shared__ T X[8 * P3], t1[8 * P3];
    __shared__ T Cm[2 * P * P];
    __shared__ int32_t ch[8];
    const int tid = threadIdx.x;
    const int64_t J = blockIdx.x;
    for (int i = tid; i < 2 * P * P; i += NT) Cm[i] = (T)C01[i];
    if (tid < 8) ch[tid] = child8[J * 8 + tid];
    __syncthreads();
    for (int i = tid; i < 8 * P3; i += NT) {
        const int c = i / P3, r = i - c * P3;
        const int q = ch[c];
        X[i] = q >= 0 ? in[(int64_t)q * P3 + r] : T(0);
    }
    __syncthreads();
    // x: t1[c][z][y][d] = sum_x C_cx[d][x] X[c][z][y][x]
    for (int i = tid; i < 8 * P3; i += NT) {
        const int d = i % P, rest = i / P, c = i / P3;
        const T* m = Cm + (c & 1) * P * P + d * P;
        const T* row = X + rest * P;
        T s = T(0);
#pragma unroll
        for (int x = 0; x < P; ++x) s += m[x] * row[x];
        t1[i] = s;
    }
    __syncthreads();
    // y: X[c][z][b][d] = sum_y C_cy[b][y] t1[c][z][y][d]
    for (int i = tid; i < 8 * P3; i += NT) {
        const int d = i % P, bb = (i / P) % P, cz = i / (P * P), c = i / P3;
        const T* m = Cm + ((c >> 1) & 1) * P * P + bb * P;
        T s = T(0);
#pragma unroll
        for (int y = 0; y < P; ++y) s += m[y] * t1[(cz * P + y) * P + d];
        X[i] = s;
    }
    __syncthreads();
    // z and the sum over children: out[a][b][d] = sum_c sum_z C_cz[a][z] X[c][z][b][d]
    for (int i = tid; i < P3; i += NT) {
        const int bd = i % (P * P), a = i / (P * P);
        T s = T(0);
        for (int c = 0; c < 8; ++c) {
            if (ch[c] < 0) continue;
            const T* m = Cm + ((c >> 2) & 1) * P * P + a * P;
#pragma unroll
            for (int z = 0; z < P; ++z) s += m[z] * X[c * P3 + z * P * P + bd];
        }
        out[J * P3 + i] = s;
    }
}

// ------------------------------------------------------------------ parent -> children
// U is the down-pass value type (double or float-float).
template <typename U, int P>
__global__ void __launch_bounds__(kDownThreads)
    k_interp_down(const U* __restrict__ par, const int32_t* __restrict__ child8, const double* __restrict__ C01,
                  U* __restrict__ io) {
    constexpr int P3 = P * P * P;
    __shared__ U X[P3], t1[2 * P3], t2[4 * P3];
    __shared__ U Ct[2 * P * P];  // Ct_c[k][m] = C_c[m][k]
    __shared__ int32_t ch[8];
    const int tid = threadIdx.x;
    const int64_t J = blockIdx.x;
    for (int i = tid; i < 2 * P * P; i += kDownThreads) {
        const int c = i / (P * P), r = i % (P * P), k = r / P, m = r % P;
        Ct[i] = U(C01[c * P * P + m * P + k]);
    }
    if (tid < 8) ch[tid] = child8[J * 8 + tid];
    for (int i = tid; i < P3; i += kDownThreads) X[i] = par[J * P3 + i];
    __syncthreads();
    // x for both cx: t1[cx][a][b][x'] = sum_d Ct_cx[x'][d] X[a][b][d]
    for (int i = tid; i < 2 * P3; i += kDownThreads) {
        const int xo = i % P, ab = (i / P) % (P * P), cx = i / P3;
        const U* m = Ct + cx * P * P + xo * P;
        const U* row = X + ab * P;
        U s = U(0);
#pragma unroll
        for (int d = 0; d < P; ++d) s += m[d] * row[d];
        t1[i] = s;
    }
    __syncthreads();
    // y for both cy: t2[cy][cx][a][y'][x'] = sum_b Ct_cy[y'][b] t1[cx][a][b][x']
    for (int i = tid; i < 4 * P3; i += kDownThreads) {
        const int xo = i % P, yo = (i / P) % P, a = (i / (P * P)) % P, cx = (i / P3) & 1, cy = i / (2 * P3);
        const U* m = Ct + cy * P * P + yo * P;
        const U* src = t1 + cx * P3 + a * P * P + xo;
        U s = U(0);
#pragma unroll
        for (int bb = 0; bb < P; ++bb) s += m[bb] * src[bb * P];
        t2[i] = s;
    }
    __syncthreads();
    // z per child, accumulate into the child's node values
    for (int i = tid; i < 8 * P3; i += kDownThreads) {
        const int r = i % P3, c = i / P3;
        const int q = ch[c];
        if (q < 0) continue;
        const int yx = r % (P * P), zo = r / (P * P);
        const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
        const U* m = Ct + cz * P * P + zo * P;
        const U* src = t2 + (cy * 2 + cx) * P3 + yx;
        U s = U(0);
#pragma unroll
        for (int a = 0; a < P; ++a) s += m[a] * src[a * P * P];
        U* dst = io + (int64_t)q * P3 + r;
        *dst = *dst + s;
    }
}

// ------------------------------------------------------------------ one (parent, child) per workgroup
// (every P = 17 level, and the Interp of levels with few parents at any P)
// The kernels above hold 8 children, or a parent's 2 + 4 partial passes, in LDS (629 /
// 275 KB at P = 17).  Here one workgroup handles one (parent, child) pair, which also
// gives levels with few parents eight times the workgroups:
//   Reg up:      k_reg_up_part writes each child's contribution to `part` (scratch), then
//                k_reg_up_sum adds them in child order c = 0..7 (as one workgroup would);
//   Interp down: each child accumulates its own values (no two workgroups write one child).
template <typename T, int P>
__global__ void __launch_bounds__(kInterpThreads)
    k_reg_up_part(const T* __restrict__ in, const int32_t* __restrict__ child8, const double* __restrict__ C01,
                  T* __restrict__ part) {
    constexpr int P3 = P * P * P;
    __shared__ T X[P3], t1[P3];
    __shared__ T Cm[2 * P * P];
    const int tid = threadIdx.x;
    const int64_t J = blockIdx.x >> 3;
    const int c = blockIdx.x & 7;
    const int q = child8[J * 8 + c];  // uniform
    if (q < 0) return;
    for (int i = tid; i < 2 * P * P; i += kInterpThreads) Cm[i] = (T)C01[i];
    for (int i = tid; i < P3; i += kInterpThreads) X[i] = in[(int64_t)q * P3 + i];
    __syncthreads();
    for (int i = tid; i < P3; i += kInterpThreads) {  // x: t1[z][y][d]
        const int d = i % P, rest = i / P;
        const T* m = Cm + (c & 1) * P * P + d * P;
        const T* row = X + rest * P;
        T sum = T(0);
#pragma unroll
        for (int x = 0; x < P; ++x) sum += m[x] * row[x];
        t1[i] = sum;
    }
    __syncthreads();
    for (int i = tid; i < P3; i += kInterpThreads) {  // y: X[z][b][d]
        const int d = i % P, bb = (i / P) % P, z = i / (P * P);
        const T* m = Cm + ((c >> 1) & 1) * P * P + bb * P;
        T sum = T(0);
#pragma unroll
        for (int y = 0; y < P; ++y) sum += m[y] * t1[(z * P + y) * P + d];
        X[i] = sum;
    }
    __syncthreads();
    T* o = part + (J * 8 + c) * P3;
    for (int i = tid; i < P3; i += kInterpThreads) {  // z
        const int bd = i % (P * P), a = i / (P * P);
        const T* m = Cm + ((c >> 2) & 1) * P * P + a * P;
        T sum = T(0);
#pragma unroll
        for (int z = 0; z < P; ++z) sum += m[z] * X[z * P * P + bd];
        o[i] = sum;
    }
}

template <typename T, int P>
__global__ void __launch_bounds__(kInterpThreads)
    k_reg_up_sum(const T* __restrict__ part, const int32_t* __restrict__ child8, T* __restrict__ out, int64_t np) {
    constexpr int P3 = P * P * P;
    const int64_t g = (int64_t)blockIdx.x * kInterpThreads + threadIdx.x;
    if (g >= np * P3) return;
    const int64_t J = g / P3;
    const int i = (int)(g - J * P3);
    T acc = T(0);
    for (int c = 0; c < 8; ++c)
        if (child8[J * 8 + c] >= 0) acc += part[(J * 8 + c) * P3 + i];
    out[g] = acc;
}

template <typename U, int P>
__global__ void __launch_bounds__(kDownThreads)
    k_interp_down_one(const U* __restrict__ par, const int32_t* __restrict__ child8, const double* __restrict__ C01,
                      U* __restrict__ io) {
    constexpr int P3 = P * P * P;
    __shared__ U X[P3], t1[P3], t2[P3];
    __shared__ U Ct[2 * P * P];  // Ct_c[k][m] = C_c[m][k]
    const int tid = threadIdx.x;
    const int64_t J = blockIdx.x >> 3;
    const int c = blockIdx.x & 7;
    const int q = child8[J * 8 + c];  // uniform
    if (q < 0) return;
    const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
    for (int i = tid; i < 2 * P * P; i += kDownThreads) {
        const int cc = i / (P * P), r = i % (P * P), k = r / P, m = r % P;
        Ct[i] = U(C01[cc * P * P + m * P + k]);
    }
    for (int i = tid; i < P3; i += kDownThreads) X[i] = par[J * P3 + i];
    __syncthreads();
    for (int i = tid; i < P3; i += kDownThreads) {  // x: t1[a][b][x']
        const int xo = i % P, ab = i / P;
        const U* m = Ct + cx * P * P + xo * P;
        const U* row = X + ab * P;
        U sum = U(0);
#pragma unroll
        for (int d = 0; d < P; ++d) sum += m[d] * row[d];
        t1[i] = sum;
    }
    __syncthreads();
    for (int i = tid; i < P3; i += kDownThreads) {  // y: t2[a][y'][x']
        const int xo = i % P, yo = (i / P) % P, a = i / (P * P);
        const U* m = Ct + cy * P * P + yo * P;
        const U* src = t1 + a * P * P + xo;
        U sum = U(0);
#pragma unroll
        for (int bb = 0; bb < P; ++bb) sum += m[bb] * src[bb * P];
        t2[i] = sum;
    }
    __syncthreads();
    for (int i = tid; i < P3; i += kDownThreads) {  // z, accumulated into the child
        const int yx = i % (P * P), zo = i / (P * P);
        const U* m = Ct + cz * P * P + zo * P;
        U sum = U(0);
#pragma unroll
        for (int a = 0; a < P; ++a) sum += m[a] * t2[a * P * P + yx];
        U* dst = io + (int64_t)q * P3 + i;
        *dst = *dst + sum;
    }
}

// Level-1 node values of the lattice scheme (p = n + 1 nodes on the grid points, Reg the
// identity on n^3 and a zero last plane): a padded copy, out[b] = [f[b]; 0] in each axis.
template <typename T>
__global__ void k_pad_copy(const T* __restrict__ f, T* __restrict__ out, int64_t nb, int n, int p) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p3 = (int64_t)p * p * p;
    if (g >= nb * p3) return;
    const int64_t b = g / p3;
    const int r = (int)(g - b * p3);
    const int x = r % p, y = (r / p) % p, z = r / (p * p);
    out[g] = (x < n && y < n && z < n) ? f[((b * n + z) * n + y) * n + x] : T(0);
}

// ------------------------------------------------------------------ level 1 -> block, FP64 add-back
template <typename T, typename U, int N, int P>
__global__ void __launch_bounds__(kBlockThreads)
    k_final(const T* vnear, const U* __restrict__ ut, const double* __restrict__ A, T* u,
            const int32_t* __restrict__ l1map, const int32_t* __restrict__ near_flag) {
    constexpr int N3 = N * N * N, P3 = P * P * P, PR = P + 1;
    // rows read at several indices at once by a wave are padded to P + 1 values (LDS banks)
    __shared__ double X[P * P * PR], t1[P * P * N], t2[P * N * N];
    __shared__ double At[N * PR];  // At[j][k] = A[k][j]
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    for (int i = tid; i < N * P; i += kBlockThreads) {
        const int jj = i / P, k = i % P;
        At[jj * PR + k] = A[k * N + jj];
    }
    const int64_t q = l1map ? (int64_t)l1map[b] : b;  // level-1 interval of this block
    for (int i = tid; i < P3; i += kBlockThreads) X[(i / P) * PR + i % P] = to_double(ut[q * P3 + i]);
    __syncthreads();
    for (int i = tid; i < P * P * N; i += kBlockThreads) {  // x: t1[a][c][x]
        const int x = i % N, ac = i / N;
        const double* m = At + x * PR;
        const double* row = X + ac * PR;
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < P; ++d) acc += m[d] * row[d];
        t1[i] = acc;
    }
    __syncthreads();
    for (int i = tid; i < P * N * N; i += kBlockThreads) {  // y: t2[a][y][x]
        const int x = i % N, y = (i / N) % N, a = i / (N * N);
        const double* m = At + y * PR;
        const double* col = t1 + a * P * N + x;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < P; ++c) acc += m[c] * col[c * N];
        t2[i] = acc;
    }
    __syncthreads();
    const T* v = vnear + b * N3;
    const bool has_near = !near_flag || near_flag[b];  // no near field: v is not read
    T* o = u + b * N3;
    for (int i = tid; i < N3; i += kBlockThreads) {  // z: u[z][y][x]
        const int yx = i % (N * N), z = i / (N * N);
        const double* m = At + z * PR;
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < P; ++a) acc += m[a] * t2[a * N * N + yx];
        o[i] = (T)((has_near ? (double)v[i] : 0.0) + acc);
    }
}

// ------------------------------------------------------------------ launchers
// (n, p) -> compile-time kernel: n in {4, 6, 8, 12, 16}, p in [2, 10], and (12, 13), (16, 17)
template <template <int, int> class K, typename... Args>
static hipError_t dispatch_np(int n, int p, Args... args) {
#define LGF_NP(NN)                                          \
    switch (p) {                                            \
        case 2: return K<NN, 2>::run(args...);              \
        case 3: return K<NN, 3>::run(args...);              \
        case 4: return K<NN, 4>::run(args...);              \
        case 5: return K<NN, 5>::run(args...);              \
        case 6: return K<NN, 6>::run(args...);              \
        case 7: return K<NN, 7>::run(args...);              \
        case 8: return K<NN, 8>::run(args...);              \
        case 9: return K<NN, 9>::run(args...);              \
        case 10: return K<NN, 10>::run(args...);            \
        default: return hipErrorInvalidValue;               \
    }
    switch (n) {
        case 4: LGF_NP(4)
        case 6: LGF_NP(6)
        case 8: LGF_NP(8)
        case 12:
            if (p == 13) return K<12, 13>::run(args...);  // the lattice scheme n_I = n + 1
            LGF_NP(12)
        case 16:
            if (p == 17) return K<16, 17>::run(args...);
            LGF_NP(16)
        default: return hipErrorInvalidValue;
    }
#undef LGF_NP
}

template <typename T>
struct RegBlockRun {
    template <int N, int P>
    struct K {
        static hipError_t run(const T* f, const double* A, T* out, int64_t nb, hipStream_t s) {
            return lgf_launch(k_reg_block<T, N, P>, dim3((unsigned)nb), dim3(kBlockThreads), 0, s, f, A, out);
        }
    };
};

template <typename T, typename U>
struct FinalRun {
    template <int N, int P>
    struct K {
        static hipError_t run(const T* vnear, const U* ut, const double* A, T* u, int64_t nb, const int32_t* l1map,
                              const int32_t* near_flag, hipStream_t s) {
            return lgf_launch(k_final<T, U, N, P>, dim3((unsigned)nb), dim3(kBlockThreads), 0, s, vnear, ut, A, u,
                              l1map, near_flag);
        }
    };
};

template <typename T>
hipError_t launch_reg_block(const T* f, const double* A, T* out, int64_t nb, int n, int p, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    return dispatch_np<RegBlockRun<T>::template K>(n, p, f, A, out, nb, s);
}

template <typename T, int P>
static hipError_t reg_up_p(const T* in, const int32_t* child8, const double* C01, T* out, int64_t np, hipStream_t s) {
    return lgf_launch(k_reg_up<T, P>, dim3((unsigned)np), dim3(kRegUpThreads), 0, s, in, child8, C01, out);
}

// Tiles of more than n_max nodes: one workgroup per (parent, child) writes each child's
// contribution to scratch, a second kernel adds them in child order (eight children of so
// many nodes do not fit one workgroup's LDS).
template <typename T, int P>
static hipError_t reg_up_parts(const T* in, const int32_t* child8, const double* C01, T* out, int64_t np,
                               hipStream_t s, void* scratch) {
    constexpr int P3 = P * P * P;
    if (!scratch) return hipErrorInvalidValue;
    const hipError_t e = lgf_launch(k_reg_up_part<T, P>, dim3((unsigned)(np * 8)), dim3(kInterpThreads), 0, s, in,
                                    child8, C01, (T*)scratch);
    if (e != hipSuccess) return e;
    return lgf_launch(k_reg_up_sum<T, P>, dim3((unsigned)((np * P3 + kInterpThreads - 1) / kInterpThreads)),
                      dim3(kInterpThreads), 0, s, (const T*)scratch, child8, out, np);
}

template <typename T>
hipError_t launch_reg_up(const T* in, const int32_t* child8, const double* C01, T* out, int64_t np, int p,
                         hipStream_t s, void* scratch) {
    if (np <= 0) return hipSuccess;
    switch (p) {
        case 2: return reg_up_p<T, 2>(in, child8, C01, out, np, s);
        case 3: return reg_up_p<T, 3>(in, child8, C01, out, np, s);
        case 4: return reg_up_p<T, 4>(in, child8, C01, out, np, s);
        case 5: return reg_up_p<T, 5>(in, child8, C01, out, np, s);
        case 6: return reg_up_p<T, 6>(in, child8, C01, out, np, s);
        case 7: return reg_up_p<T, 7>(in, child8, C01, out, np, s);
        case 8: return reg_up_p<T, 8>(in, child8, C01, out, np, s);
        case 9: return reg_up_p<T, 9>(in, child8, C01, out, np, s);
        case 10: return reg_up_p<T, 10>(in, child8, C01, out, np, s);
        case 13: return reg_up_parts<T, 13>(in, child8, C01, out, np, s, scratch);
        case 17: return reg_up_parts<T, 17>(in, child8, C01, out, np, s, scratch);
        default: return hipErrorInvalidValue;
    }
}

template <typename U, int P>
static hipError_t interp_down_p(const U* par, const int32_t* child8, const double* C01, U* io, int64_t np,
                                hipStream_t s) {
    // levels with few parents: one workgroup per (parent, child), eight times the
    // workgroups (the same sums in the same order, so the same bits as one per parent)
    if (np <= 256)
        return lgf_launch(k_interp_down_one<U, P>, dim3((unsigned)(np * 8)), dim3(kDownThreads), 0, s, par, child8,
                          C01, io);
    return lgf_launch(k_interp_down<U, P>, dim3((unsigned)np), dim3(kDownThreads), 0, s, par, child8, C01, io);
}

template <typename U>
hipError_t launch_interp_down(const U* par, const int32_t* child8, const double* C01, U* io, int64_t nparent,
                              int p, hipStream_t s) {
    if (nparent <= 0) return hipSuccess;
    switch (p) {
        case 2: return interp_down_p<U, 2>(par, child8, C01, io, nparent, s);
        case 3: return interp_down_p<U, 3>(par, child8, C01, io, nparent, s);
        case 4: return interp_down_p<U, 4>(par, child8, C01, io, nparent, s);
        case 5: return interp_down_p<U, 5>(par, child8, C01, io, nparent, s);
        case 6: return interp_down_p<U, 6>(par, child8, C01, io, nparent, s);
        case 7: return interp_down_p<U, 7>(par, child8, C01, io, nparent, s);
        case 8: return interp_down_p<U, 8>(par, child8, C01, io, nparent, s);
        case 9: return interp_down_p<U, 9>(par, child8, C01, io, nparent, s);
        case 10: return interp_down_p<U, 10>(par, child8, C01, io, nparent, s);
        case 13:
            return lgf_launch(k_interp_down_one<U, 13>, dim3((unsigned)(nparent * 8)), dim3(kDownThreads), 0, s, par,
                              child8, C01, io);
        case 17:
            return lgf_launch(k_interp_down_one<U, 17>, dim3((unsigned)(nparent * 8)), dim3(kDownThreads), 0, s, par,
                              child8, C01, io);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_pad_copy(const T* f, T* out, int64_t nb, int n, int p, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    const int64_t tot = nb * (int64_t)p * p * p;
    return lgf_launch(k_pad_copy<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, f, out, nb, n, p);
}

template <typename T, typename U>
hipError_t launch_final(const T* vnear, const U* ut, const double* A, T* u, int64_t nb, int n, int p, hipStream_t s,
                        const int32_t* l1map, const int32_t* near_flag) {
    if (nb <= 0) return hipSuccess;
    return dispatch_np<FinalRun<T, U>::template K>(n, p, vnear, ut, A, u, nb, l1map, near_flag, s);
}

template hipError_t launch_reg_block<double>(const double*, const double*, double*, int64_t, int, int, hipStream_t);
template hipError_t launch_pad_copy<double>(const double*, double*, int64_t, int, int, hipStream_t);
template hipError_t launch_pad_copy<float>(const float*, float*, int64_t, int, int, hipStream_t);
template hipError_t launch_reg_block<float>(const float*, const double*, float*, int64_t, int, int, hipStream_t);
template hipError_t launch_reg_up<double>(const double*, const int32_t*, const double*, double*, int64_t, int,
                                         hipStream_t, void*);
template hipError_t launch_reg_up<float>(const float*, const int32_t*, const double*, float*, int64_t, int,
                                         hipStream_t, void*);
template hipError_t launch_interp_down<double>(const double*, const int32_t*, const double*, double*, int64_t, int,
                                               hipStream_t);
template hipError_t launch_interp_down<ff32>(const ff32*, const int32_t*, const double*, ff32*, int64_t, int,
                                             hipStream_t);
template hipError_t launch_final<double, double>(const double*, const double*, const double*, double*, int64_t, int,
                                                 int, hipStream_t, const int32_t*, const int32_t*);
template hipError_t launch_final<float, ff32>(const float*, const ff32*, const double*, float*, int64_t, int, int,
                                              hipStream_t, const int32_t*, const int32_t*);

}  // namespace lgfdev
