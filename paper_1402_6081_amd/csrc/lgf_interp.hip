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
constexpr int kMaxN = 16, kMaxP = 10;

// ------------------------------------------------------------------ block -> level 1
template <typename T>
__global__ void __launch_bounds__(kInterpThreads)
    k_reg_block(const T* __restrict__ f, const double* __restrict__ A, T* __restrict__ out, int n, int p) {
    __shared__ T t1[kMaxN * kMaxN * kMaxP], t2[kMaxN * kMaxP * kMaxP];
    __shared__ T Am[kMaxP * kMaxN];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int n3 = n * n * n, p3 = p * p * p;
    for (int i = tid; i < p * n; i += kInterpThreads) Am[i] = (T)A[i];
    __syncthreads();
    const T* X = f + b * n3;
    // x: t1[z][y][d] = sum_x A[d][x] f[z][y][x]  (rows read straight from HBM)
    for (int i = tid; i < n * n * p; i += kInterpThreads) {
        const int d = i % p, zy = i / p;
        const T* row = X + zy * n;
        const T* m = Am + d * n;
        T s = T(0);
        for (int x = 0; x < n; ++x) s += m[x] * row[x];
        t1[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < n * p * p; i += kInterpThreads) {  // y: t2[z][c][d]
        const int d = i % p, c = (i / p) % p, z = i / (p * p);
        const T* m = Am + c * n;
        T s = T(0);
        for (int y = 0; y < n; ++y) s += m[y] * t1[(z * n + y) * p + d];
        t2[i] = s;
    }
    __syncthreads();
    T* o = out + b * p3;
    for (int i = tid; i < p3; i += kInterpThreads) {  // z: out[a][c][d]
        const int cd = i % (p * p), a = i / (p * p);
        const T* m = Am + a * n;
        T s = T(0);
        for (int z = 0; z < n; ++z) s += m[z] * t2[z * (p * p) + cd];
        o[i] = s;
    }
}

// ------------------------------------------------------------------ children -> parent
template <typename T, int P>
__global__ void __launch_bounds__(kInterpThreads)
    k_reg_up(const T* __restrict__ in, const int32_t* __restrict__ child8, const double* __restrict__ C01,
             T* __restrict__ out) {
    constexpr int P3 = P * P * P;
    __shared__ T X[8 * P3], t1[8 * P3];
    __shared__ T Cm[2 * P * P];
    __shared__ int32_t ch[8];
    const int tid = threadIdx.x;
    const int64_t J = blockIdx.x;
    for (int i = tid; i < 2 * P * P; i += kInterpThreads) Cm[i] = (T)C01[i];
    if (tid < 8) ch[tid] = child8[J * 8 + tid];
    __syncthreads();
    for (int i = tid; i < 8 * P3; i += kInterpThreads) {
        const int c = i / P3, r = i - c * P3;
        const int q = ch[c];
        X[i] = q >= 0 ? in[(int64_t)q * P3 + r] : T(0);
    }
    __syncthreads();
    // x: t1[c][z][y][d] = sum_x C_cx[d][x] X[c][z][y][x]
    for (int i = tid; i < 8 * P3; i += kInterpThreads) {
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
    for (int i = tid; i < 8 * P3; i += kInterpThreads) {
        const int d = i % P, bb = (i / P) % P, cz = i / (P * P), c = i / P3;
        const T* m = Cm + ((c >> 1) & 1) * P * P + bb * P;
        T s = T(0);
#pragma unroll
        for (int y = 0; y < P; ++y) s += m[y] * t1[(cz * P + y) * P + d];
        X[i] = s;
    }
    __syncthreads();
    // z and the sum over children: out[a][b][d] = sum_c sum_z C_cz[a][z] X[c][z][b][d]
    for (int i = tid; i < P3; i += kInterpThreads) {
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
__global__ void __launch_bounds__(kInterpThreads)
    k_interp_down(const U* __restrict__ par, const int32_t* __restrict__ child8, const double* __restrict__ C01,
                  U* __restrict__ io) {
    constexpr int P3 = P * P * P;
    __shared__ U X[P3], t1[2 * P3], t2[4 * P3];
    __shared__ U Ct[2 * P * P];  // Ct_c[k][m] = C_c[m][k]
    __shared__ int32_t ch[8];
    const int tid = threadIdx.x;
    const int64_t J = blockIdx.x;
    for (int i = tid; i < 2 * P * P; i += kInterpThreads) {
        const int c = i / (P * P), r = i % (P * P), k = r / P, m = r % P;
        Ct[i] = U(C01[c * P * P + m * P + k]);
    }
    if (tid < 8) ch[tid] = child8[J * 8 + tid];
    for (int i = tid; i < P3; i += kInterpThreads) X[i] = par[J * P3 + i];
    __syncthreads();
    // x for both cx: t1[cx][a][b][x'] = sum_d Ct_cx[x'][d] X[a][b][d]
    for (int i = tid; i < 2 * P3; i += kInterpThreads) {
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
    for (int i = tid; i < 4 * P3; i += kInterpThreads) {
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
    for (int i = tid; i < 8 * P3; i += kInterpThreads) {
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

// ------------------------------------------------------------------ level 1 -> block, FP64 add-back
template <typename T, typename U>
__global__ void __launch_bounds__(kInterpThreads)
    k_final(const T* vnear, const U* __restrict__ ut, const double* __restrict__ A, T* u, int n, int p) {
    __shared__ double X[kMaxP * kMaxP * kMaxP], t1[kMaxP * kMaxP * kMaxN], t2[kMaxP * kMaxN * kMaxN];
    __shared__ double At[kMaxN * kMaxP];  // At[j][k] = A[k][j]
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int n3 = n * n * n, p3 = p * p * p;
    for (int i = tid; i < n * p; i += kInterpThreads) {
        const int j = i / p, k = i % p;
        At[i] = A[k * n + j];
    }
    for (int i = tid; i < p3; i += kInterpThreads) X[i] = to_double(ut[b * p3 + i]);
    __syncthreads();
    for (int i = tid; i < p * p * n; i += kInterpThreads) {  // x: t1[a][c][x]
        const int x = i % n, ac = i / n;
        const double* m = At + x * p;
        const double* row = X + ac * p;
        double s = 0.0;
        for (int d = 0; d < p; ++d) s += m[d] * row[d];
        t1[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < p * n * n; i += kInterpThreads) {  // y: t2[a][y][x]
        const int x = i % n, y = (i / n) % n, a = i / (n * n);
        const double* m = At + y * p;
        double s = 0.0;
        for (int c = 0; c < p; ++c) s += m[c] * t1[(a * p + c) * n + x];
        t2[i] = s;
    }
    __syncthreads();
    const T* v = vnear + b * n3;
    T* o = u + b * n3;
    for (int i = tid; i < n3; i += kInterpThreads) {  // z: u[z][y][x]
        const int yx = i % (n * n), z = i / (n * n);
        const double* m = At + z * p;
        double s = 0.0;
        for (int a = 0; a < p; ++a) s += m[a] * t2[a * n * n + yx];
        o[i] = (T)((double)v[i] + s);
    }
}

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_reg_block(const T* f, const double* A, T* out, int64_t nb, int n, int p, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reg_block<T>, dim3((unsigned)nb), dim3(kInterpThreads), 0, s, f, A, out, n, p);
    return hipGetLastError();
}

template <typename T, int P>
static hipError_t reg_up_p(const T* in, const int32_t* child8, const double* C01, T* out, int64_t np, hipStream_t s) {
    hipLaunchKernelGGL((k_reg_up<T, P>), dim3((unsigned)np), dim3(kInterpThreads), 0, s, in, child8, C01, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reg_up(const T* in, const int32_t* child8, const double* C01, T* out, int64_t np, int p,
                         hipStream_t s) {
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
        default: return hipErrorInvalidValue;
    }
}

template <typename U, int P>
static hipError_t interp_down_p(const U* par, const int32_t* child8, const double* C01, U* io, int64_t np,
                                hipStream_t s) {
    hipLaunchKernelGGL((k_interp_down<U, P>), dim3((unsigned)np), dim3(kInterpThreads), 0, s, par, child8, C01, io);
    return hipGetLastError();
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
        default: return hipErrorInvalidValue;
    }
}

template <typename T, typename U>
hipError_t launch_final(const T* vnear, const U* ut, const double* A, T* u, int64_t nb, int n, int p, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_final<T, U>), dim3((unsigned)nb), dim3(kInterpThreads), 0, s, vnear, ut, A, u, n, p);
    return hipGetLastError();
}

template hipError_t launch_reg_block<double>(const double*, const double*, double*, int64_t, int, int, hipStream_t);
template hipError_t launch_reg_block<float>(const float*, const double*, float*, int64_t, int, int, hipStream_t);
template hipError_t launch_reg_up<double>(const double*, const int32_t*, const double*, double*, int64_t, int,
                                          hipStream_t);
template hipError_t launch_reg_up<float>(const float*, const int32_t*, const double*, float*, int64_t, int,
                                         hipStream_t);
template hipError_t launch_interp_down<double>(const double*, const int32_t*, const double*, double*, int64_t, int,
                                               hipStream_t);
template hipError_t launch_interp_down<ff32>(const ff32*, const int32_t*, const double*, ff32*, int64_t, int,
                                             hipStream_t);
template hipError_t launch_final<double, double>(const double*, const double*, const double*, double*, int64_t, int,
                                                 int, hipStream_t);
template hipError_t launch_final<float, ff32>(const float*, const ff32*, const double*, float*, int64_t, int, int,
                                              hipStream_t);

}  // namespace lgfdev
