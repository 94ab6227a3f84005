// Level interactions (Step 2 of Sec. 3.1, Eq. alg_mult):
//   uhat^P = sum_{Q in InflList(P)} Prod(fhat^Q, khat^{P-Q})
// computed independently for every DFT coefficient.  One thread owns one coefficient
// of one target; the list of P is uniform across the workgroup, so list entries are
// scalar loads and the fhat / khat streams are contiguous across lanes.
#include "lgf_internal.h"

namespace lgfdev {

constexpr int kProdThreads = 256;

// Level 0: the near-neighbour list is dense: nbr[P][27] holds the index of block
// P - D (or -1), D = (d % 3 - 1, (d / 3) % 3 - 1, d / 9 - 1).
template <typename T>
__global__ void __launch_bounds__(kProdThreads)
    k_prod_near(const cplx<T>* __restrict__ fhat, const cplx<T>* __restrict__ khat,
                const int32_t* __restrict__ nbr, cplx<T>* __restrict__ uhat, int S) {
    const int w = blockIdx.y * kProdThreads + threadIdx.x;
    const int64_t P = blockIdx.x;
    if (w >= S) return;
    const int32_t* nb = nbr + P * 27;
    T ar = T(0), ai = T(0);
#pragma unroll 3
    for (int d = 0; d < 27; ++d) {
        const int q = nb[d];
        if (q < 0) continue;
        const cplx<T> f = fhat[(int64_t)q * S + w];
        const cplx<T> k = khat[(int64_t)d * S + w];
        ar += f.x * k.x - f.y * k.y;
        ai += f.x * k.y + f.y * k.x;
    }
    uhat[P * S + w] = cplx<T>{ar, ai};
}

// Levels >= 1: CSR interaction lists (ptr, src, off) with off indexing the level's spectra.
template <typename T>
__global__ void __launch_bounds__(kProdThreads)
    k_prod_far(const cplx<T>* __restrict__ fhat, const cplx<T>* __restrict__ khat,
               const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
               const int32_t* __restrict__ off, cplx<T>* __restrict__ uhat, int S) {
    const int w = blockIdx.y * kProdThreads + threadIdx.x;
    const int64_t P = blockIdx.x;
    if (w >= S) return;
    const int e0 = ptr[P], e1 = ptr[P + 1];
    T ar = T(0), ai = T(0);
    for (int e = e0; e < e1; ++e) {
        const int q = src[e];
        const int o = off[e];
        const cplx<T> f = fhat[(int64_t)q * S + w];
        const cplx<T> k = khat[(int64_t)o * S + w];
        ar += f.x * k.x - f.y * k.y;
        ai += f.x * k.y + f.y * k.x;
    }
    uhat[P * S + w] = cplx<T>{ar, ai};
}

template <typename T>
hipError_t launch_prod_near(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* nbr, cplx<T>* uhat,
                            int64_t ntarget, int S, hipStream_t s) {
    if (ntarget <= 0) return hipSuccess;
    dim3 grid((unsigned)ntarget, (unsigned)((S + kProdThreads - 1) / kProdThreads));
    hipLaunchKernelGGL(k_prod_near<T>, grid, dim3(kProdThreads), 0, s, fhat, khat, nbr, uhat, S);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prod_far(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* ptr, const int32_t* src,
                           const int32_t* off, cplx<T>* uhat, int64_t ntarget, int S, hipStream_t s) {
    if (ntarget <= 0) return hipSuccess;
    dim3 grid((unsigned)ntarget, (unsigned)((S + kProdThreads - 1) / kProdThreads));
    hipLaunchKernelGGL(k_prod_far<T>, grid, dim3(kProdThreads), 0, s, fhat, khat, ptr, src, off, uhat, S);
    return hipGetLastError();
}

template hipError_t launch_prod_near<double>(const cplx<double>*, const cplx<double>*, const int32_t*,
                                             cplx<double>*, int64_t, int, hipStream_t);
template hipError_t launch_prod_near<float>(const cplx<float>*, const cplx<float>*, const int32_t*,
                                            cplx<float>*, int64_t, int, hipStream_t);
template hipError_t launch_prod_far<double>(const cplx<double>*, const cplx<double>*, const int32_t*,
                                            const int32_t*, const int32_t*, cplx<double>*, int64_t, int,
                                            hipStream_t);
template hipError_t launch_prod_far<float>(const cplx<float>*, const cplx<float>*, const int32_t*,
                                           const int32_t*, const int32_t*, cplx<float>*, int64_t, int,
                                           hipStream_t);

}  // namespace lgfdev
