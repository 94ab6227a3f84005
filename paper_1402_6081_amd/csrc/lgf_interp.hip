// Regularization (Reg, Eq. alg_reg / kcprss1) and interpolation (Interp, Eq. alg_interp
// / kcprss3) between levels, as tensor products of 1D Lagrange matrices (Sec. 2.5):
//   block -> level-1 interval   ftilde = (A x A x A) f           A[k][j] = phi_k(j (p-1)/n)
//   children -> parent          ftilde_J = sum_c (C_c x C_c x C_c) ftilde_{2J+c}
//                                                                 C_c[m][k] = phi_m((c(p-1)+k)/2)
//   parent -> child (add)       utilde_{2J+c} += (C_c^T x C_c^T x C_c^T) utilde_J
//   level-1 interval -> block   u = vnear + (A^T x A^T x A^T) utilde    (FP64 add-back)
// One workgroup per block/interval; each 3D product is three 1D passes through LDS.
#include "lgf_internal.h"

namespace lgfdev {

constexpr int kInterpThreads = 256;
constexpr int kMaxN = 16, kMaxP = 10;
constexpr int kBufA = kMaxN * kMaxN * kMaxN;  // largest tile
constexpr int kBufB = kMaxN * kMaxN * kMaxP;  // largest intermediate

// out[a][c][d] = sum Mz[a][z] My[c][y] Mx[d][x] X[z][y][x]; matrices row-major [o][i].
// X, t1, t2 in LDS; `emit(index, value)` receives the output.
template <typename Acc, typename Emit>
__device__ __forceinline__ void tensor3(const Acc* X, int iz, int iy, int ix, const Acc* Mz, const Acc* My,
                                        const Acc* Mx, int oz, int oy, int ox, Acc* t1, Acc* t2, Emit emit) {
    const int tid = threadIdx.x;
    for (int i = tid; i < iz * iy * ox; i += kInterpThreads) {
        const int d = i % ox, zy = i / ox;
        const Acc* row = X + zy * ix;
        const Acc* m = Mx + d * ix;
        Acc s = Acc(0);
        for (int x = 0; x < ix; ++x) s += m[x] * row[x];
        t1[i] = s;  // [z][y][d]
    }
    __syncthreads();
    for (int i = tid; i < iz * oy * ox; i += kInterpThreads) {
        const int d = i % ox, c = (i / ox) % oy, z = i / (ox * oy);
        const Acc* m = My + c * iy;
        Acc s = Acc(0);
        for (int y = 0; y < iy; ++y) s += m[y] * t1[(z * iy + y) * ox + d];
        t2[i] = s;  // [z][c][d]
    }
    __syncthreads();
    for (int i = tid; i < oz * oy * ox; i += kInterpThreads) {
        const int cd = i % (oy * ox), a = i / (oy * ox);
        const Acc* m = Mz + a * iz;
        Acc s = Acc(0);
        for (int z = 0; z < iz; ++z) s += m[z] * t2[z * (oy * ox) + cd];
        emit(i, s);
    }
}

template <typename T>
__global__ void __launch_bounds__(kInterpThreads)
    k_reg_block(const T* __restrict__ f, const double* __restrict__ A, T* __restrict__ out, int n, int p) {
    __shared__ T X[kBufA], t1[kBufB], t2[kBufB];
    __shared__ T Am[kMaxP * kMaxN];
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int n3 = n * n * n, p3 = p * p * p;
    for (int i = tid; i < p * n; i += kInterpThreads) Am[i] = (T)A[i];
    for (int i = tid; i < n3; i += kInterpThreads) X[i] = f[b * n3 + i];
    __syncthreads();
    T* o = out + b * p3;
    tensor3<T>(X, n, n, n, Am, Am, Am, p, p, p, t1, t2, [&](int i, T v) { o[i] = v; });
}

template <typename T>
__global__ void __launch_bounds__(kInterpThreads)
    k_reg_up(const T* __restrict__ in, const int32_t* __restrict__ child8, const double* __restrict__ C01,
             T* __restrict__ out, int p) {
    __shared__ T X[kMaxP * kMaxP * kMaxP], acc[kMaxP * kMaxP * kMaxP];
    __shared__ T t1[kMaxP * kMaxP * kMaxP], t2[kMaxP * kMaxP * kMaxP];
    __shared__ T Cm[2 * kMaxP * kMaxP];
    const int tid = threadIdx.x;
    const int64_t J = blockIdx.x;
    const int p3 = p * p * p;
    for (int i = tid; i < 2 * p * p; i += kInterpThreads) Cm[i] = (T)C01[i];
    for (int i = tid; i < p3; i += kInterpThreads) acc[i] = T(0);
    __syncthreads();
    for (int c = 0; c < 8; ++c) {
        const int q = child8[J * 8 + c];
        if (q < 0) continue;  // uniform across the workgroup
        for (int i = tid; i < p3; i += kInterpThreads) X[i] = in[(int64_t)q * p3 + i];
        __syncthreads();
        const T* Cx = Cm + (c & 1) * p * p;
        const T* Cy = Cm + ((c >> 1) & 1) * p * p;
        const T* Cz = Cm + ((c >> 2) & 1) * p * p;
        tensor3<T>(X, p, p, p, Cz, Cy, Cx, p, p, p, t1, t2, [&](int i, T v) { acc[i] += v; });
        __syncthreads();
    }
    for (int i = tid; i < p3; i += kInterpThreads) out[J * p3 + i] = acc[i];
}

template <typename T>
__global__ void __launch_bounds__(kInterpThreads)
    k_interp_down(const T* __restrict__ par, const int32_t* __restrict__ parent, const int32_t* __restrict__ cpos,
                  const double* __restrict__ C01, T* __restrict__ io, int p) {
    __shared__ T X[kMaxP * kMaxP * kMaxP], t1[kMaxP * kMaxP * kMaxP], t2[kMaxP * kMaxP * kMaxP];
    __shared__ T Ct[2 * kMaxP * kMaxP];  // transposed: Ct_c[k][m] = C_c[m][k]
    const int tid = threadIdx.x;
    const int64_t i0 = blockIdx.x;
    const int p3 = p * p * p;
    for (int i = tid; i < 2 * p * p; i += kInterpThreads) {
        const int c = i / (p * p), r = i % (p * p), k = r / p, m = r % p;
        Ct[i] = (T)C01[c * p * p + m * p + k];
    }
    const int J = parent[i0];
    const int c = cpos[i0];
    for (int i = tid; i < p3; i += kInterpThreads) X[i] = par[(int64_t)J * p3 + i];
    __syncthreads();
    const T* Cx = Ct + (c & 1) * p * p;
    const T* Cy = Ct + ((c >> 1) & 1) * p * p;
    const T* Cz = Ct + ((c >> 2) & 1) * p * p;
    T* o = io + i0 * p3;
    tensor3<T>(X, p, p, p, Cz, Cy, Cx, p, p, p, t1, t2, [&](int i, T v) { o[i] += v; });
}

template <typename T>
__global__ void __launch_bounds__(kInterpThreads)
    k_final(const T* vnear, const T* __restrict__ ut, const double* __restrict__ A, T* u, int n, int p) {
    __shared__ double X[kMaxP * kMaxP * kMaxP], t1[kBufB], t2[kBufB];
    __shared__ double At[kMaxN * kMaxP];  // At[j][k] = A[k][j]
    const int tid = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int n3 = n * n * n, p3 = p * p * p;
    for (int i = tid; i < n * p; i += kInterpThreads) {
        const int j = i / p, k = i % p;
        At[i] = A[k * n + j];
    }
    for (int i = tid; i < p3; i += kInterpThreads) X[i] = (double)ut[b * p3 + i];
    __syncthreads();
    const T* v = vnear + b * n3;
    T* o = u + b * n3;
    tensor3<double>(X, p, p, p, At, At, At, n, n, n, t1, t2, [&](int i, double s) { o[i] = (T)((double)v[i] + s); });
}

template <typename T>
hipError_t launch_reg_block(const T* f, const double* A, T* out, int64_t nb, int n, int p, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reg_block<T>, dim3((unsigned)nb), dim3(kInterpThreads), 0, s, f, A, out, n, p);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_reg_up(const T* in, const int32_t* child8, const double* C01, T* out, int64_t nparent, int p,
                         hipStream_t s) {
    if (nparent <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reg_up<T>, dim3((unsigned)nparent), dim3(kInterpThreads), 0, s, in, child8, C01, out, p);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_interp_down(const T* par, const int32_t* parent, const int32_t* cpos, const double* C01, T* io,
                              int64_t nchild, int p, hipStream_t s) {
    if (nchild <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_interp_down<T>, dim3((unsigned)nchild), dim3(kInterpThreads), 0, s, par, parent, cpos, C01,
                       io, p);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_final(const T* vnear, const T* ut, const double* A, T* u, int64_t nb, int n, int p, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_final<T>, dim3((unsigned)nb), dim3(kInterpThreads), 0, s, vnear, ut, A, u, n, p);
    return hipGetLastError();
}

#define LGF_INST(T)                                                                                            \
    template hipError_t launch_reg_block<T>(const T*, const double*, T*, int64_t, int, int, hipStream_t);      \
    template hipError_t launch_reg_up<T>(const T*, const int32_t*, const double*, T*, int64_t, int,            \
                                         hipStream_t);                                                         \
    template hipError_t launch_interp_down<T>(const T*, const int32_t*, const int32_t*, const double*, T*,     \
                                              int64_t, int, hipStream_t);                                      \
    template hipError_t launch_final<T>(const T*, const T*, const double*, T*, int64_t, int, int, hipStream_t);
LGF_INST(double)
LGF_INST(float)
#undef LGF_INST

}  // namespace lgfdev
