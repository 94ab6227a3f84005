// Level interactions (Step 2 of Sec. 3.1, Eq. alg_mult):
//   uhat^P = sum_{Q in InflList(P)} Prod(fhat^Q, khat^{P-Q}),
// independently for every DFT coefficient.
//
// Source spectra arrays hold one extra, all-zero item (index = item count) that stands in
// for inactive neighbours, so the inner loops load without branches or selects.
// Both blocked kernels exploit the lattice structure of the lists: the 8 targets that
// share a parent J see the same candidate sources (level 0: the 4^3 blocks 2J-1..2J+2;
// levels >= 1: the 6^3 children of the 27 neighbours of J) at offsets D = P - Q that
// depend only on the two child positions.  Each source spectrum is therefore read once per
// group instead of once per (target, source) pair, and the kernel spectra of a frequency
// chunk sit in an LDS tile shared by the workgroup (27 offsets at level 0, the 343 offsets
// of [-3, 3]^3 at levels >= 1).
// A plain CSR kernel covers the top level of a truncated tree, whose list is "every
// non-adjacent interval" and has no such structure.
#include "lgf_internal.h"

namespace lgfdev {

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Both
// blocked kernels map a 1D grid so that XCD x processes whole frequency chunks
// {c : c % 8 == x}, walking every group of such a chunk back to back: all reuse of a source
// spectrum within a chunk then stays in one L2.  Returns false for padding workgroups.
constexpr int kXcds = 8;
__device__ __forceinline__ bool xcd_tile(int nchunks, int ngroupblocks, int& chunk, int& gblock) {
    const int L = blockIdx.x;
    const int xcd = L % kXcds, k = L / kXcds;
    chunk = (k / ngroupblocks) * kXcds + xcd;
    gblock = k % ngroupblocks;
    return chunk < nchunks;
}
__host__ __forceinline__ unsigned xcd_grid(int nchunks, int ngroupblocks) {
    const int padded = (nchunks + kXcds - 1) / kXcds * kXcds;
    return (unsigned)padded * (unsigned)ngroupblocks;
}

// complex multiply-accumulate as four FMAs
template <typename T>
__device__ __forceinline__ void cmac(T& ar, T& ai, const cplx<T>& f, const cplx<T>& k) {
    ar = fma(f.x, k.x, ar);
    ar = fma(-f.y, k.y, ar);
    ai = fma(f.x, k.y, ai);
    ai = fma(f.y, k.x, ai);
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------------ level 0
// Groups g: tgt8[g][c] = block 2J + c (c = cx | cy<<1 | cz<<2) or -1;
// src64[g][s] = block 2J + (sx-1, sy-1, sz-1), s = sx + 4 sy + 16 sz, or the zero sentinel
// item (index nb) when that block is not active.  fhat holds nb + 1 items (the last is 0).
// One wave = 64 consecutive frequencies of one group; the 4 waves of a workgroup share the
// frequency chunk and its kernel tile in LDS.  The tile has rows for dz in [-2, 2] (the
// rows with |dz| = 2 are zero) so the source-slab loop needs no branches.
template <typename T, int kNearWaves>
__global__ void __launch_bounds__(64 * kNearWaves)
    k_prod_near_grouped(const cplx<T>* __restrict__ fhat, const cplx<T>* __restrict__ khat,
                        const int32_t* __restrict__ tgt8, const int32_t* __restrict__ src64,
                        cplx<T>* __restrict__ uhat, int S, int ngroups, int nb) {
    __shared__ cplx<T> tile[45 * 64];  // row (dx+1) + 3 (dy+1) + 9 (dz+2)
    const int lane = threadIdx.x & 63;
    int chunk, gb;
    if (!xcd_tile(S / 64, (ngroups + kNearWaves - 1) / kNearWaves, chunk, gb)) return;
    const int w0 = chunk * 64;
    const int w = w0 + lane;  // frequency (S is a multiple of 64)
    for (int i = threadIdx.x; i < 45 * 64; i += 64 * kNearWaves) {
        const int r = i >> 6, dz = r / 9 - 2;
        tile[i] = (dz < -1 || dz > 1) ? cplx<T>{T(0), T(0)} : khat[spec_at(r - 9, w0 + (i & 63), 27)];
    }
    __syncthreads();
    const int g = wave_uniform(gb * kNearWaves + (threadIdx.x >> 6));
    if (g >= ngroups) return;
    T ar[8], ai[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        ar[c] = T(0);
        ai[c] = T(0);
    }
    const int32_t* sg = src64 + (int64_t)g * 64;
    const cplx<T>* fl = fhat + (int64_t)chunk * (nb + 1) * 64 + lane;  // this lane's frequency
#pragma unroll 1
    for (int sz = 0; sz < 4; ++sz) {  // source z slab; x and y unrolled
        cplx<T> f[16];
#pragma unroll
        for (int sxy = 0; sxy < 16; ++sxy) f[sxy] = fl[(int64_t)sg[sz * 16 + sxy] * 64];
        // dz = cz - (sz - 1) in [-2, 2]; row base for cz = 0 and cz = 1
        const cplx<T>* t0 = tile + (9 * (3 - sz)) * 64 + lane;
        const cplx<T>* t1 = tile + (9 * (4 - sz)) * 64 + lane;
#pragma unroll
        for (int sxy = 0; sxy < 16; ++sxy) {
            const int sx = (sxy & 3) - 1, sy = (sxy >> 2) - 1;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int dx = (c & 1) - sx, dy = ((c >> 1) & 1) - sy;
                if (dx < -1 || dx > 1 || dy < -1 || dy > 1) continue;  // compile-time
                const cplx<T> k = ((c >> 2) ? t1 : t0)[((dx + 1) + 3 * (dy + 1)) * 64];
                cmac(ar[c], ai[c], f[sxy], k);
            }
        }
    }
    const int32_t* tg = tgt8 + (int64_t)g * 8;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int t = tg[c];
        if (t >= 0) uhat[spec_at(t, w, nb)] = cplx<T>{ar[c], ai[c]};
    }
}

// ------------------------------------------------------------------ levels >= 1, sibling blocked
// Parents J (level l+1): src216[J][e * 8 + cs] = level-l interval 2(J + e') + cs with
// e' = (ex-1, ey-1, ez-1), e = ex + 3 ey + 9 ez, or the zero sentinel item (index nitems);
// child8[J][c] = target 2J + c (or -1).  khat: 343 offsets, id (Dx+3) + 7 (Dy+3) + 49 (Dz+3).
// Lane = (child c, frequency j of a chunk of 8); one wave per parent, the waves of a
// workgroup share the [343][8] kernel tile in LDS.  The 8 child lanes of a frequency read
// the same source coefficient, so each source spectrum is fetched once per parent.
constexpr int kFarWC = 8;
constexpr int kFarRow = kFarWC + 1;  // padded tile row (breaks LDS bank aliasing between rows)
// Tile layout: row ((3 - Dx) + 7 (3 - Dy) + 49 (3 - Dz)), column j holds khat^D at frequency
// w0 + j, and 0 for the 27 offsets with |D|_inf <= 1 (not interaction-list offsets).  With
// D = c - cs - 2e the row is base(c, e) + (csx + 7 csy + 49 csz): a compile-time offset for
// the unrolled source child cs, and near pairs add exact zeros.
template <typename T, int kFarWaves>
__global__ void __launch_bounds__(64 * kFarWaves)
    k_prod_far_sib(const cplx<T>* __restrict__ fhat, const cplx<T>* __restrict__ khat,
                   const int32_t* __restrict__ child8, const int32_t* __restrict__ src216,
                   cplx<T>* __restrict__ uhat, int S, int nparents, int nitems) {
    __shared__ cplx<T> tile[343 * kFarRow];
    const int nchunks = (S + kFarWC - 1) / kFarWC;
    int chunk, pb;
    if (!xcd_tile(nchunks, (nparents + kFarWaves - 1) / kFarWaves, chunk, pb)) return;
    const int w0 = chunk * kFarWC;
    for (int i = threadIdx.x; i < 343 * kFarWC; i += 64 * kFarWaves) {
        const int r = i / kFarWC, j = i - r * kFarWC;
        const int Dx = 3 - r % 7, Dy = 3 - (r / 7) % 7, Dz = 3 - r / 49;
        const int o = (Dx + 3) + 7 * (Dy + 3) + 49 * (Dz + 3);
        const bool near = Dx >= -1 && Dx <= 1 && Dy >= -1 && Dy <= 1 && Dz >= -1 && Dz <= 1;
        tile[r * kFarRow + j] = (w0 + j < S && !near) ? khat[spec_at(o, w0 + j, 343)] : cplx<T>{T(0), T(0)};
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int c = lane >> 3, j = lane & 7;
    const int w = w0 + j;
    const bool live = w < S;
    const int J = wave_uniform(pb * kFarWaves + (threadIdx.x >> 6));
    if (J >= nparents) return;
    const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
    // this lane's frequency column of the source spectra (padding lanes read column w0)
    const cplx<T>* fl = fhat + (int64_t)((live ? w : w0) >> 6) * (nitems + 1) * 64 + ((live ? w : w0) & 63);
    const int32_t* sj = src216 + (int64_t)J * 216;
    T ar = T(0), ai = T(0);
    // double-buffered: the 8 source loads of neighbour e+1 are in flight while e is consumed
    cplx<T> fa[8], fb[8];
#pragma unroll
    for (int cs = 0; cs < 8; ++cs) fa[cs] = fl[(int64_t)sj[cs] * 64];
#pragma unroll 1
    for (int e = 0; e < 27; e += 2) {
        if (e + 1 < 27) {
#pragma unroll
            for (int cs = 0; cs < 8; ++cs) fb[cs] = fl[(int64_t)sj[(e + 1) * 8 + cs] * 64];
        }
        {
            const int ex = e % 3 - 1, ey = (e / 3) % 3 - 1, ez = e / 9 - 1;
            const cplx<T>* kb = tile + ((3 - cx + 2 * ex) + 7 * (3 - cy + 2 * ey) + 49 * (3 - cz + 2 * ez)) * kFarRow + j;
#pragma unroll
            for (int cs = 0; cs < 8; ++cs)
                cmac(ar, ai, fa[cs], kb[((cs & 1) + 7 * ((cs >> 1) & 1) + 49 * (cs >> 2)) * kFarRow]);
        }
        if (e + 1 >= 27) break;
        if (e + 2 < 27) {
#pragma unroll
            for (int cs = 0; cs < 8; ++cs) fa[cs] = fl[(int64_t)sj[(e + 2) * 8 + cs] * 64];
        }
        {
            const int e1 = e + 1;
            const int ex = e1 % 3 - 1, ey = (e1 / 3) % 3 - 1, ez = e1 / 9 - 1;
            const cplx<T>* kb = tile + ((3 - cx + 2 * ex) + 7 * (3 - cy + 2 * ey) + 49 * (3 - cz + 2 * ez)) * kFarRow + j;
#pragma unroll
            for (int cs = 0; cs < 8; ++cs)
                cmac(ar, ai, fb[cs], kb[((cs & 1) + 7 * ((cs >> 1) & 1) + 49 * (cs >> 2)) * kFarRow]);
        }
    }
    const int t = child8[(int64_t)J * 8 + c];
    if (t >= 0 && live) uhat[spec_at(t, w, nitems)] = cplx<T>{ar, ai};
}

// ------------------------------------------------------------------ generic CSR (top level)
constexpr int kProdThreads = 256;

// Targets tgt[i] (i = blockIdx.x) with list entries [ptr[i], ptr[i+1]).
template <typename T>
__global__ void __launch_bounds__(kProdThreads)
    k_prod_far(const cplx<T>* __restrict__ fhat, const cplx<T>* __restrict__ khat,
               const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
               const int32_t* __restrict__ off, const int32_t* __restrict__ tgt, cplx<T>* __restrict__ uhat, int S,
               int nitems, int noff) {
    const int w = blockIdx.y * kProdThreads + threadIdx.x;
    const int64_t i = blockIdx.x;
    if (w >= S) return;
    const int64_t P = tgt[i];
    const int e0 = ptr[i], e1 = ptr[i + 1];
    T ar = T(0), ai = T(0);
    for (int e = e0; e < e1; ++e) {
        const int q = src[e];
        const int o = off[e];
        const cplx<T> f = fhat[spec_at(q, w, nitems + 1)];
        const cplx<T> k = khat[spec_at(o, w, noff)];
        cmac(ar, ai, f, k);
    }
    uhat[spec_at(P, w, nitems)] = cplx<T>{ar, ai};
}

template <typename T, int NW>
static hipError_t near_nw(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* tgt8, const int32_t* src64,
                          cplx<T>* uhat, int64_t ngroups, int64_t nitems, int S, hipStream_t s) {
    const unsigned grid = xcd_grid(S / 64, (int)((ngroups + NW - 1) / NW));
    hipLaunchKernelGGL((k_prod_near_grouped<T, NW>), dim3(grid), dim3(64 * NW), 0, s, fhat, khat, tgt8, src64, uhat, S,
                       (int)ngroups, (int)nitems);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prod_near(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* tgt8, const int32_t* src64,
                            cplx<T>* uhat, int64_t ngroups, int64_t nitems, int S, int waves, hipStream_t s) {
    if (ngroups <= 0) return hipSuccess;
    if (S % 64) return hipErrorInvalidValue;
    switch (waves) {
        case 2: return near_nw<T, 2>(fhat, khat, tgt8, src64, uhat, ngroups, nitems, S, s);
        case 8: return near_nw<T, 8>(fhat, khat, tgt8, src64, uhat, ngroups, nitems, S, s);
        default: return near_nw<T, 4>(fhat, khat, tgt8, src64, uhat, ngroups, nitems, S, s);
    }
}

template <typename T, int NW>
static hipError_t far_nw(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* child8, const int32_t* src216,
                         cplx<T>* uhat, int64_t nparents, int64_t nitems, int S, hipStream_t s) {
    const unsigned grid = xcd_grid((S + kFarWC - 1) / kFarWC, (int)((nparents + NW - 1) / NW));
    hipLaunchKernelGGL((k_prod_far_sib<T, NW>), dim3(grid), dim3(64 * NW), 0, s, fhat, khat, child8, src216, uhat, S,
                       (int)nparents, (int)nitems);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prod_far_sib(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* child8,
                               const int32_t* src216, cplx<T>* uhat, int64_t nparents, int64_t nitems, int S,
                               int waves, hipStream_t s) {
    if (nparents <= 0) return hipSuccess;
    switch (waves) {
        case 4: return far_nw<T, 4>(fhat, khat, child8, src216, uhat, nparents, nitems, S, s);
        case 16: return far_nw<T, 16>(fhat, khat, child8, src216, uhat, nparents, nitems, S, s);
        default: return far_nw<T, 8>(fhat, khat, child8, src216, uhat, nparents, nitems, S, s);
    }
}

template <typename T>
hipError_t launch_prod_far(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* ptr, const int32_t* src,
                           const int32_t* off, const int32_t* tgt, cplx<T>* uhat, int64_t ntgt, int64_t nitems,
                           int noff, int S, hipStream_t s) {
    if (ntgt <= 0) return hipSuccess;
    dim3 grid((unsigned)ntgt, (unsigned)((S + kProdThreads - 1) / kProdThreads));
    hipLaunchKernelGGL(k_prod_far<T>, grid, dim3(kProdThreads), 0, s, fhat, khat, ptr, src, off, tgt, uhat, S,
                       (int)nitems, noff);
    return hipGetLastError();
}

#define LGF_INST(T)                                                                                              \
    template hipError_t launch_prod_near<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*,      \
                                            cplx<T>*, int64_t, int64_t, int, int, hipStream_t);                  \
    template hipError_t launch_prod_far_sib<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*,   \
                                               cplx<T>*, int64_t, int64_t, int, int, hipStream_t);               \
    template hipError_t launch_prod_far<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*,       \
                                           const int32_t*, const int32_t*, cplx<T>*, int64_t, int64_t, int, int, \
                                           hipStream_t);
LGF_INST(double)
LGF_INST(float)
#undef LGF_INST

}  // namespace lgfdev
