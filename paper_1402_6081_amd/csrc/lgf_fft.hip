// Zero-padded forward FFT (Pad + FFT, Eq. alg_upfft) and truncated inverse FFT
// (FFT^-1 + Trunc, Eq. alg_dwfft) of one block or interval per workgroup.
//
// Data: an m^3 real tile [z][y][x] <-> its padded M^3 real-to-complex spectrum
// [kz][ky][kx], M = 2m, kx in [0, M/2], stored chunk-major (spec_at) across the batch.
// One workgroup per tile; the tile lives in a [z < m][ky < M][kx <= M/2] LDS array (the
// largest intermediate of either direction), the real input/output is staged in the
// not-yet-used upper ky half of each z plane so that HBM reads and writes are fully
// coalesced.  The staged rows are padded to m + 1 values: the x pass reads (and the
// inverse writes) one row per lane, and rows m apart would share LDS banks.  Passes: x (real rows), y (complex
// columns of the z < m planes), z (complex columns, straight to/from HBM).
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "lgf_device.h"
#include "lgf_internal.h"

namespace lgfdev {

// One launch may transform several levels' tiles (segments of the grid with their own
// input, output and output item count; one workgroup per item).
template <typename T>
struct FwdSegs {
    const T* in[kMaxFarSegs];
    cplx<T>* out[kMaxFarSegs];
    int64_t nout[kMaxFarSegs];
    int64_t start[kMaxFarSegs];
    int n;
};

// Persistent: a workgroup transforms tiles blockIdx.x, blockIdx.x + gridDim.x, ... of the
// launch; while it transforms one, the next tile's input is already on its way into
// registers (a tile occupies so much LDS that at most one or two workgroups share a CU, so
// the input reads would otherwise stall the CU).
template <typename T, int m, int M, int NT>
__global__ void __launch_bounds__(NT) k_pad_fft(const FwdSegs<T> segs, int64_t total) {
    constexpr int H = M / 2 + 1;
    constexpr int PLANE = M * H;
    constexpr int NPRE = (m * m * m + NT - 1) / NT;
    static_assert(M == 2 * m, "padded length is twice the tile edge");
    __shared__ cplx<T> buf[m * PLANE];
    const int tid = threadIdx.x;
    // tile vb of the launch: its segment (uniform selects over the kernel arguments) and
    // its index b within the segment
    auto locate = [&](int64_t vb, const T*& in, cplx<T>*& out, int64_t& nout, int64_t& b) {
        in = segs.in[0];
        out = segs.out[0];
        nout = segs.nout[0];
        int64_t b0 = 0;
#pragma unroll
        for (int k = 1; k < kMaxFarSegs; ++k)
            if (k < segs.n && vb >= segs.start[k]) {
                in = segs.in[k];
                out = segs.out[k];
                nout = segs.nout[k];
                b0 = segs.start[k];
            }
        b = vb - b0;
    };
    auto fetch = [&](int64_t vb, T(&pre)[NPRE]) {
        const T* in;
        cplx<T>* o;
        int64_t no, b;
        locate(vb, in, o, no, b);
        const T* src = in + (size_t)b * (m * m * m);
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int i = tid + k * NT;
            pre[k] = i < m * m * m ? src[i] : T(0);
        }
    };
    int64_t vb = blockIdx.x;
    if (vb >= total) return;
    T pre[NPRE];
    fetch(vb, pre);
    for (; vb < total; vb += gridDim.x) {
        const T* in;
        cplx<T>* out;
        int64_t nout, bi;
        locate(vb, in, out, nout, bi);
        const size_t b = (size_t)bi;
        // stage the real tile: plane z -> upper ky half of LDS plane z
#pragma unroll
        for (int k = 0; k < NPRE; ++k) {
            const int i = tid + k * NT;
            if (i < m * m * m) {
                const int z = i / (m * m), r = i - z * (m * m);
                reinterpret_cast<T*>(buf + z * PLANE + m * H)[(r / m) * (m + 1) + r % m] = pre[k];
            }
        }
        __syncthreads();
        if (vb + gridDim.x < total) fetch(vb + gridDim.x, pre);  // the next tile's input
        // x pass: real rows (z, y) -> kx in [0, M/2]
        for (int row = tid; row < m * m; row += NT) {
            const int z = row / m, y = row - z * m;
            const T* s = reinterpret_cast<const T*>(buf + z * PLANE + m * H) + y * (m + 1);
            cplx<T>* d = buf + z * PLANE + y * H;
            T xr[m];
#pragma unroll
            for (int j = 0; j < m; ++j) xr[j] = s[j];
            if constexpr (is_pow2(M)) {
                T xi[m], Xr[M], Xi[M];
#pragma unroll
                for (int j = 0; j < m; ++j) xi[j] = T(0);
                pencil_fwd<T, m, M>(xr, xi, Xr, Xi);
#pragma unroll
                for (int k = 0; k < H; ++k) d[k] = cplx<T>{Xr[k], Xi[k]};
            } else {
                T Xr[H], Xi[H];
                pencil_r2c<T, m, M>(xr, Xr, Xi);
#pragma unroll
                for (int k = 0; k < H; ++k) d[k] = cplx<T>{Xr[k], Xi[k]};
            }
        }
        __syncthreads();
        // y pass: columns (z, kx), y < m -> ky < M
        for (int col = tid; col < m * H; col += NT) {
            const int z = col / H, kx = col - z * H;
            cplx<T>* base = buf + z * PLANE + kx;
            T xr[m], xi[m];
#pragma unroll
            for (int j = 0; j < m; ++j) {
                const cplx<T> v = base[j * H];
                xr[j] = v.x;
                xi[j] = v.y;
            }
            T Xr[M], Xi[M];
            pencil_fwd<T, m, M>(xr, xi, Xr, Xi);
#pragma unroll
            for (int k = 0; k < M; ++k) base[k * H] = cplx<T>{Xr[k], Xi[k]};
        }
        __syncthreads();
        // z pass: columns (ky, kx), z < m -> kz < M, written to HBM (chunk-major spectrum)
        for (int col = tid; col < PLANE; col += NT) {
            T xr[m], xi[m];
#pragma unroll
            for (int j = 0; j < m; ++j) {
                const cplx<T> v = buf[j * PLANE + col];
                xr[j] = v.x;
                xi[j] = v.y;
            }
            T Xr[M], Xi[M];
            pencil_fwd<T, m, M>(xr, xi, Xr, Xi);
#pragma unroll
            for (int k = 0; k < M; ++k) out[spec_at(b, k * PLANE + col, nout)] = cplx<T>{Xr[k], Xi[k]};
        }
        __syncthreads();  // the next tile is staged into buf
    }
}

// Inverse: spectrum elements of type Tin, arithmetic in A, real output of type Tout.
// (FP64 path: all double.  FP32 path: float at level 0 and at level 1 of the lattice
// scheme; at the other levels >= 1 the float spectra are inverted in double arithmetic and
// written as float-float node values (each double rounded to a hi + lo float pair).  The
// float-float arithmetic instantiation A = ff32 is kept for tiles up to 10 nodes.)
// One launch may invert several levels' spectra (segments of the grid with their own
// input, output and item count; one workgroup per item).
template <typename Tin, typename Tout>
struct InvSegs {
    const cplx<Tin>* in[kMaxFarSegs];
    Tout* out[kMaxFarSegs];
    int64_t nbatch[kMaxFarSegs];
    int64_t start[kMaxFarSegs];
    int n;
};

template <typename Tin, typename A, typename Tout, int m, int M, int NT>
__global__ void __launch_bounds__(NT) k_ifft_trunc(const InvSegs<Tin, Tout> segs, const int32_t* __restrict__ out_map,
                                                   int opitch) {
    constexpr int H = M / 2 + 1;
    constexpr int PLANE = M * H;
    static_assert(M == 2 * m, "padded length is twice the tile edge");
    __shared__ cplx<A> buf[m * PLANE];
    const int tid = threadIdx.x;
    // this workgroup's segment (uniform selects over the kernel arguments)
    const cplx<Tin>* __restrict__ in = segs.in[0];
    Tout* __restrict__ out = segs.out[0];
    int64_t nbatch = segs.nbatch[0], b0 = 0;
#pragma unroll
    for (int k = 1; k < kMaxFarSegs; ++k)
        if (k < segs.n && (int64_t)blockIdx.x >= segs.start[k]) {
            in = segs.in[k];
            out = segs.out[k];
            nbatch = segs.nbatch[k];
            b0 = segs.start[k];
        }
    const size_t b = (size_t)((int64_t)blockIdx.x - b0);

    // z pass: HBM columns (ky, kx), kz < M -> z < m
    for (int col = tid; col < PLANE; col += NT) {
        A Xr[M], Xi[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const cplx<Tin> v = in[spec_at(b, k * PLANE + col, nbatch)];
            Xr[k] = A(v.x);
            Xi[k] = A(v.y);
        }
        A xr[m], xi[m];
        pencil_inv<A, m, M>(Xr, Xi, xr, xi);
#pragma unroll
        for (int j = 0; j < m; ++j) buf[j * PLANE + col] = cplx<A>{xr[j], xi[j]};
    }
    __syncthreads();
    // y pass: columns (z, kx), ky < M -> y < m
    for (int col = tid; col < m * H; col += NT) {
        const int z = col / H, kx = col - z * H;
        cplx<A>* base = buf + z * PLANE + kx;
        A Xr[M], Xi[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const cplx<A> v = base[k * H];
            Xr[k] = v.x;
            Xi[k] = v.y;
        }
        A xr[m], xi[m];
        pencil_inv<A, m, M>(Xr, Xi, xr, xi);
#pragma unroll
        for (int j = 0; j < m; ++j) base[j * H] = cplx<A>{xr[j], xi[j]};
    }
    __syncthreads();
    // x pass: Hermitian rows (z, y) -> real x < m, staged in the upper ky half
    for (int row = tid; row < m * m; row += NT) {
        const int z = row / m, y = row - z * m;
        const cplx<A>* s = buf + z * PLANE + y * H;
        A Yr[H], Yi[H];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const cplx<A> v = s[k];
            Yr[k] = v.x;
            Yi[k] = v.y;
        }
        A x[m];
        pencil_c2r<A, m, M>(Yr, Yi, x);
        A* d = reinterpret_cast<A*>(buf + z * PLANE + m * H) + y * (m + 1);
#pragma unroll
        for (int j = 0; j < m; ++j) d[j] = x[j];
    }
    __syncthreads();
    // output tiles of opitch^3 values: the m^3 results, zeros in the planes beyond them
    Tout* dst = out + (out_map ? (size_t)out_map[b] : b) * (size_t)(opitch * opitch * opitch);
    if (opitch == m) {
        for (int i = tid; i < m * m * m; i += NT) {
            const int z = i / (m * m), r = i - z * (m * m);
            dst[i] = (Tout)reinterpret_cast<const A*>(buf + z * PLANE + m * H)[(r / m) * (m + 1) + r % m];
        }
    } else {
        for (int i = tid; i < opitch * opitch * opitch; i += NT) {
            const int x = i % opitch, y = (i / opitch) % opitch, z = i / (opitch * opitch);
            dst[i] = (z < m && y < m && x < m) ? (Tout)reinterpret_cast<const A*>(buf + z * PLANE + m * H)[y * (m + 1) + x]
                                               : Tout(0);
        }
    }
}

// ------------------------------------------------------------------ two-phase transforms
constexpr int kShare = 3;  // threads sharing one pencil (each forms every third output)
// For tiles whose one-workgroup LDS tile [m][M][M/2+1] exceeds the 160 KB of a workgroup
// (m = 17: 166 KB of complex doubles), the transforms run in two kernels through an HBM
// intermediate [z < m][ky < M][kx <= M/2] per item (`scratch`, complex of 16 bytes):
//   forward  k_fft2_xy (per z plane: x pass, y pass -> scratch), k_fft2_z (z pass -> spectrum);
//   inverse  k_ifft2_z (z pass -> scratch), k_ifft2_yx (per z plane: y pass, x pass -> tile).
template <typename T, int m, int M, int NT>
__global__ void __launch_bounds__(NT) k_fft2_xy(const T* __restrict__ in, cplx<T>* __restrict__ scratch) {
    // one workgroup per z plane of an item: the x and y passes do not mix planes
    constexpr int H = M / 2 + 1;
    __shared__ T tile[m * m];
    __shared__ cplx<T> buf[m * H];  // [y][kx]
    __shared__ double2 tw[M];
    const int tid = threadIdx.x;
    const size_t b = blockIdx.x / m;
    const int z = blockIdx.x - (int)b * m;
    const T* src = in + b * (m * m * m) + z * (m * m);
    stage_roots<M>(tw, tid, NT);
    for (int i = tid; i < m * m; i += NT) tile[i] = src[i];
    __syncthreads();
    for (int t = tid; t < kShare * m; t += NT) {  // x pass: real rows, kShare threads per row
        const int y = t / kShare, k0 = t - y * kShare;
        T xr[m], xi[m];
#pragma unroll
        for (int j = 0; j < m; ++j) {
            xr[j] = tile[y * m + j];
            xi[j] = T(0);
        }
        cplx<T>* d = buf + y * H;
        dft_each<T, m, M, -1, H>(xr, xi, tw, [&](int k, T re, T im) { d[k] = cplx<T>{re, im}; }, k0, kShare);
    }
    __syncthreads();
    cplx<T>* dst = scratch + b * (m * M * H) + z * (M * H);
    for (int t = tid; t < kShare * H; t += NT) {  // y pass: columns kx -> [ky][kx] of plane z
        const int kx = t / kShare, k0 = t - kx * kShare;
        T xr[m], xi[m];
#pragma unroll
        for (int j = 0; j < m; ++j) {
            const cplx<T> v = buf[j * H + kx];
            xr[j] = v.x;
            xi[j] = v.y;
        }
        cplx<T>* d = dst + kx;
        dft_each<T, m, M, -1, M>(xr, xi, tw, [&](int k, T re, T im) { d[k * H] = cplx<T>{re, im}; }, k0, kShare);
    }
}

// z pass of the forward two-phase transform: one thread per column (ky, kx) of one item
template <typename T, int m, int M, int NT>
__global__ void __launch_bounds__(NT) k_fft2_z(const cplx<T>* __restrict__ scratch, cplx<T>* __restrict__ out,
                                               int64_t nout) {
    constexpr int H = M / 2 + 1;
    constexpr int PLANE = M * H;
    __shared__ double2 tw[M];
    stage_roots<M>(tw, threadIdx.x, NT);
    __syncthreads();
    const size_t b = blockIdx.y;
    const int t = blockIdx.x * NT + threadIdx.x;
    if (t >= kShare * PLANE) return;
    const int col = t / kShare, k0 = t - col * kShare;
    const cplx<T>* s = scratch + b * (m * PLANE) + col;
    T xr[m], xi[m];
#pragma unroll
    for (int j = 0; j < m; ++j) {
        const cplx<T> v = s[j * PLANE];
        xr[j] = v.x;
        xi[j] = v.y;
    }
    dft_each<T, m, M, -1, M>(
        xr, xi, tw, [&](int k, T re, T im) { out[spec_at(b, k * PLANE + col, nout)] = cplx<T>{re, im}; }, k0,
        kShare);
}

// z pass of the inverse two-phase transform: spectrum (Tin) -> scratch (arithmetic type A)
template <typename Tin, typename A, int m, int M, int NT>
__global__ void __launch_bounds__(NT) k_ifft2_z(const cplx<Tin>* __restrict__ in, cplx<A>* __restrict__ scratch,
                                                int64_t nbatch) {
    constexpr int H = M / 2 + 1;
    constexpr int PLANE = M * H;
    __shared__ double2 tw[M];
    stage_roots<M>(tw, threadIdx.x, NT);
    __syncthreads();
    const size_t b = blockIdx.y;
    const int t = blockIdx.x * NT + threadIdx.x;
    if (t >= kShare * PLANE) return;
    const int col = t / kShare, j0 = t - col * kShare;
    A Xr[M], Xi[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const cplx<Tin> v = in[spec_at(b, k * PLANE + col, nbatch)];
        Xr[k] = A(v.x);
        Xi[k] = A(v.y);
    }
    cplx<A>* d = scratch + b * (m * PLANE) + col;
    dft_each<A, M, M, +1, m>(Xr, Xi, tw, [&](int j, A re, A im) { d[j * PLANE] = cplx<A>{re, im}; }, j0, kShare);
}

// y and x passes of the inverse two-phase transform: scratch -> real tile (Tout); one
// workgroup per z plane of an item
template <typename A, typename Tout, int m, int M, int NT>
__global__ void __launch_bounds__(NT) k_ifft2_yx(const cplx<A>* __restrict__ scratch, Tout* __restrict__ out,
                                                 const int32_t* __restrict__ out_map) {
    constexpr int H = M / 2 + 1;
    __shared__ cplx<A> buf[m * H];  // [y][kx]
    __shared__ A tile[m * m];
    __shared__ double2 tw[M];
    const int tid = threadIdx.x;
    const size_t b = blockIdx.x / m;
    const int z = blockIdx.x - (int)b * m;
    const cplx<A>* s = scratch + b * (m * M * H) + z * (M * H);
    stage_roots<M>(tw, tid, NT);
    __syncthreads();
    for (int t = tid; t < kShare * H; t += NT) {  // y pass: ky < M -> y < m, kShare threads per column
        const int kx = t / kShare, j0 = t - kx * kShare;
        A Xr[M], Xi[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const cplx<A> v = s[k * H + kx];
            Xr[k] = v.x;
            Xi[k] = v.y;
        }
        cplx<A>* d = buf + kx;
        dft_each<A, M, M, +1, m>(Xr, Xi, tw, [&](int j, A re, A im) { d[j * H] = cplx<A>{re, im}; }, j0, kShare);
    }
    __syncthreads();
    for (int t = tid; t < kShare * m; t += NT) {  // x pass: Hermitian rows -> real x < m
        const int y = t / kShare, j0 = t - y * kShare;
        A Yr[H], Yi[H];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const cplx<A> v = buf[y * H + k];
            Yr[k] = v.x;
            Yi[k] = v.y;
        }
        A* d = tile + y * m;
        c2r_each<A, m, M>(Yr, Yi, tw, [&](int j, A v) { d[j] = v; }, j0, kShare);
    }
    __syncthreads();
    Tout* dst = out + (out_map ? (size_t)out_map[b] : b) * (m * m * m) + z * (m * m);
    for (int i = tid; i < m * m; i += NT) dst[i] = (Tout)tile[i];
}

template <typename T, int m>
static hipError_t fwd_two_phase(const T* in, cplx<T>* out, int64_t nbatch, int64_t nout, void* scratch,
                                hipStream_t s) {
    constexpr int M = 2 * m, PLANE = M * (M / 2 + 1), NT = 256;
    if (!scratch) return hipErrorInvalidValue;
    hipError_t e = lgf_launch(k_fft2_xy<T, m, M, 64>, dim3((unsigned)(nbatch * m)), dim3(64), 0, s, in,
                              (cplx<T>*)scratch);
    if (e != hipSuccess) return e;
    const dim3 grid((kShare * PLANE + NT - 1) / NT, (unsigned)nbatch);
    return lgf_launch(k_fft2_z<T, m, M, NT>, grid, dim3(NT), 0, s, (const cplx<T>*)scratch, out, nout);
}

template <typename Tin, typename A, typename Tout, int m>
static hipError_t inv_two_phase(const cplx<Tin>* in, Tout* out, int64_t nbatch, const int32_t* out_map,
                                void* scratch, hipStream_t s) {
    constexpr int M = 2 * m, PLANE = M * (M / 2 + 1), NT = 256;
    if (!scratch) return hipErrorInvalidValue;
    const dim3 grid((kShare * PLANE + NT - 1) / NT, (unsigned)nbatch);
    hipError_t e = lgf_launch(k_ifft2_z<Tin, A, m, M, NT>, grid, dim3(NT), 0, s, in, (cplx<A>*)scratch, nbatch);
    if (e != hipSuccess) return e;
    return lgf_launch(k_ifft2_yx<A, Tout, m, M, 64>, dim3((unsigned)(nbatch * m)), dim3(64), 0, s,
                      (const cplx<A>*)scratch, out, out_map);
}

// nt: threads per workgroup (0 = default: 256, measured faster than 128 for the small
// tiles of levels >= 1 as well); the autotuner picks among {128, 256, 512} for the level-0
// tiles (m = 8, 16).  The forward FP64 16^3 tile is not offered 512 threads: its 32-point
// pencils would then spill (the inverse's fit, 219 registers, and are its default).

// Tiles whose LDS allows at most two workgroups per CU (the level-0 tiles) get a
// persistent grid (measured: the 256^3 level-0 FP64 transform 375 -> 248 us, FP32 143 ->
// 108 us; the small level >= 1 tiles were 5% slower persistent, so they keep one
// workgroup per tile).
template <typename T, int m, int NT>
static hipError_t fwd_mnt(const FwdSegs<T>& segs, int64_t nblocks, hipStream_t s) {
    auto kernel = k_pad_fft<T, m, 2 * m, NT>;
    return lgf_launch(kernel, dim3((unsigned)persistent_grid(kernel, NT, nblocks, 2)), dim3(NT), 0, s, segs,
                      nblocks);
}

template <typename T, int m>
static hipError_t launch_fwd_segs(const FwdSegs<T>& segs, int64_t nblocks, hipStream_t s, int nt = 0) {
    if constexpr (m == 8 || m == 16) {
        if constexpr (!(m == 16 && sizeof(T) == 8))
            if (nt == 512) return fwd_mnt<T, m, 512>(segs, nblocks, s);
        if (nt == 128) return fwd_mnt<T, m, 128>(segs, nblocks, s);
    }
    return fwd_mnt<T, m, 256>(segs, nblocks, s);
}

template <typename T, int m>
static hipError_t launch_fwd_m(const T* in, cplx<T>* out, int64_t nbatch, int64_t nout, hipStream_t s,
                               int nt = 0) {
    FwdSegs<T> segs{};
    segs.in[0] = in;
    segs.out[0] = out;
    segs.nout[0] = nout;
    segs.n = 1;
    return launch_fwd_segs<T, m>(segs, nbatch, s, nt);
}

template <typename Tin, typename A, typename Tout, int m, int NT>
static hipError_t inv_mnt(const InvSegs<Tin, Tout>& segs, int64_t nblocks, const int32_t* out_map, int opitch,
                          hipStream_t s) {
    return lgf_launch(k_ifft_trunc<Tin, A, Tout, m, 2 * m, NT>, dim3((unsigned)nblocks), dim3(NT), 0, s, segs,
                      out_map, opitch);
}

template <typename Tin, typename A, typename Tout, int m>
static hipError_t launch_inv_segs(const InvSegs<Tin, Tout>& segs, int64_t nblocks, const int32_t* out_map,
                                  int opitch, hipStream_t s, int nt = 0) {
    if (opitch <= 0) opitch = m;
    // FP64 16^3 tiles default to 512 threads: one workgroup fills a CU's LDS, and 8 waves
    // keep twice the column loads in flight (256^3: 331 -> 299 us; 128^3: 51 -> 47 us)
    if (nt == 0 && m == 16 && sizeof(A) == 8) nt = 512;
    if constexpr ((m == 8 || m == 16) && !std::is_same<A, ff32>::value) {
        if (nt == 512) return inv_mnt<Tin, A, Tout, m, 512>(segs, nblocks, out_map, opitch, s);
        if (nt == 128) return inv_mnt<Tin, A, Tout, m, 128>(segs, nblocks, out_map, opitch, s);
    }
    return inv_mnt<Tin, A, Tout, m, 256>(segs, nblocks, out_map, opitch, s);
}

template <typename Tin, typename A, typename Tout, int m>
static hipError_t launch_inv_m(const cplx<Tin>* in, Tout* out, int64_t nbatch, const int32_t* out_map, int opitch,
                               hipStream_t s, int nt = 0) {
    InvSegs<Tin, Tout> segs{};
    segs.in[0] = in;
    segs.out[0] = out;
    segs.nbatch[0] = nbatch;
    segs.n = 1;
    return launch_inv_segs<Tin, A, Tout, m>(segs, nbatch, out_map, opitch, s, nt);
}

template <typename T>
hipError_t launch_pad_fft(int m, const T* in, cplx<T>* out, int64_t nbatch, hipStream_t s, int nt, int64_t nout,
                          void* scratch) {
    if (nbatch <= 0) return hipSuccess;
    if (nout <= 0) nout = nbatch + 1;
    switch (m) {
        case 17: return fwd_two_phase<T, 17>(in, out, nbatch, nout, scratch, s);
        case 2: return launch_fwd_m<T, 2>(in, out, nbatch, nout, s);
        case 3: return launch_fwd_m<T, 3>(in, out, nbatch, nout, s);
        case 4: return launch_fwd_m<T, 4>(in, out, nbatch, nout, s);
        case 5: return launch_fwd_m<T, 5>(in, out, nbatch, nout, s);
        case 6: return launch_fwd_m<T, 6>(in, out, nbatch, nout, s);
        case 7: return launch_fwd_m<T, 7>(in, out, nbatch, nout, s);
        case 8: return launch_fwd_m<T, 8>(in, out, nbatch, nout, s, nt);
        case 9: return launch_fwd_m<T, 9>(in, out, nbatch, nout, s);
        case 10: return launch_fwd_m<T, 10>(in, out, nbatch, nout, s);
        case 12: return launch_fwd_m<T, 12>(in, out, nbatch, nout, s);
        case 13: return launch_fwd_m<T, 13>(in, out, nbatch, nout, s);
        case 16: return launch_fwd_m<T, 16>(in, out, nbatch, nout, s, nt);
        default: return hipErrorInvalidValue;
    }
}

template <typename Tin, typename A, typename Tout>
hipError_t launch_ifft_trunc(int m, const cplx<Tin>* in, Tout* out, int64_t nbatch, hipStream_t s, int nt,
                             const int32_t* out_map, void* scratch, int opitch) {
    if (nbatch <= 0) return hipSuccess;
    if (opitch > 0 && opitch < m) return hipErrorInvalidValue;  // output tiles hold the m^3 results
    switch (m) {
        case 17: return inv_two_phase<Tin, A, Tout, 17>(in, out, nbatch, out_map, scratch, s);
        case 2: return launch_inv_m<Tin, A, Tout, 2>(in, out, nbatch, out_map, opitch, s);
        case 3: return launch_inv_m<Tin, A, Tout, 3>(in, out, nbatch, out_map, opitch, s);
        case 4: return launch_inv_m<Tin, A, Tout, 4>(in, out, nbatch, out_map, opitch, s);
        case 5: return launch_inv_m<Tin, A, Tout, 5>(in, out, nbatch, out_map, opitch, s);
        case 6: return launch_inv_m<Tin, A, Tout, 6>(in, out, nbatch, out_map, opitch, s);
        case 7: return launch_inv_m<Tin, A, Tout, 7>(in, out, nbatch, out_map, opitch, s);
        case 8: return launch_inv_m<Tin, A, Tout, 8>(in, out, nbatch, out_map, opitch, s, nt);
        case 9: return launch_inv_m<Tin, A, Tout, 9>(in, out, nbatch, out_map, opitch, s);
        case 10: return launch_inv_m<Tin, A, Tout, 10>(in, out, nbatch, out_map, opitch, s);
        // the large tiles (level 0 of n = 12 and 16, levels >= 1 of the 13-node scheme) are
        // not inverted in float-float arithmetic
        case 12:
            if constexpr (!std::is_same<A, ff32>::value)
                return launch_inv_m<Tin, A, Tout, 12>(in, out, nbatch, out_map, opitch, s);
            return hipErrorInvalidValue;
        case 13:
            if constexpr (!std::is_same<A, ff32>::value)
                return launch_inv_m<Tin, A, Tout, 13>(in, out, nbatch, out_map, opitch, s);
            return hipErrorInvalidValue;
        case 16:
            if constexpr (!std::is_same<A, ff32>::value)
                return launch_inv_m<Tin, A, Tout, 16>(in, out, nbatch, out_map, opitch, s, nt);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_pad_fft_levels(int m, const FwdLevel<T>* lv, int nlev, hipStream_t s) {
    if (nlev <= 0) return hipSuccess;
    if (nlev > kMaxFarSegs) return hipErrorInvalidValue;
    FwdSegs<T> segs{};
    int64_t nblocks = 0;
    for (int k = 0; k < nlev; ++k) {
        if (lv[k].nbatch <= 0) return hipErrorInvalidValue;
        segs.in[k] = lv[k].in;
        segs.out[k] = lv[k].out;
        segs.nout[k] = lv[k].nout > 0 ? lv[k].nout : lv[k].nbatch + 1;
        segs.start[k] = nblocks;
        nblocks += lv[k].nbatch;
    }
    segs.n = nlev;
    switch (m) {
        case 2: return launch_fwd_segs<T, 2>(segs, nblocks, s);
        case 3: return launch_fwd_segs<T, 3>(segs, nblocks, s);
        case 4: return launch_fwd_segs<T, 4>(segs, nblocks, s);
        case 5: return launch_fwd_segs<T, 5>(segs, nblocks, s);
        case 6: return launch_fwd_segs<T, 6>(segs, nblocks, s);
        case 7: return launch_fwd_segs<T, 7>(segs, nblocks, s);
        case 8: return launch_fwd_segs<T, 8>(segs, nblocks, s);
        case 9: return launch_fwd_segs<T, 9>(segs, nblocks, s);
        case 10: return launch_fwd_segs<T, 10>(segs, nblocks, s);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_pad_fft_levels<double>(int, const FwdLevel<double>*, int, hipStream_t);
template hipError_t launch_pad_fft_levels<float>(int, const FwdLevel<float>*, int, hipStream_t);

template <typename Tin, typename A, typename Tout>
hipError_t launch_ifft_trunc_levels(int m, const InvLevel<Tin, Tout>* lv, int nlev, hipStream_t s) {
    if (nlev <= 0) return hipSuccess;
    if (nlev > kMaxFarSegs) return hipErrorInvalidValue;
    InvSegs<Tin, Tout> segs{};
    int64_t nblocks = 0;
    for (int k = 0; k < nlev; ++k) {
        if (lv[k].nbatch <= 0) return hipErrorInvalidValue;
        segs.in[k] = lv[k].in;
        segs.out[k] = lv[k].out;
        segs.nbatch[k] = lv[k].nbatch;
        segs.start[k] = nblocks;
        nblocks += lv[k].nbatch;
    }
    segs.n = nlev;
    switch (m) {
        case 2: return launch_inv_segs<Tin, A, Tout, 2>(segs, nblocks, nullptr, 0, s);
        case 3: return launch_inv_segs<Tin, A, Tout, 3>(segs, nblocks, nullptr, 0, s);
        case 4: return launch_inv_segs<Tin, A, Tout, 4>(segs, nblocks, nullptr, 0, s);
        case 5: return launch_inv_segs<Tin, A, Tout, 5>(segs, nblocks, nullptr, 0, s);
        case 6: return launch_inv_segs<Tin, A, Tout, 6>(segs, nblocks, nullptr, 0, s);
        case 7: return launch_inv_segs<Tin, A, Tout, 7>(segs, nblocks, nullptr, 0, s);
        case 8: return launch_inv_segs<Tin, A, Tout, 8>(segs, nblocks, nullptr, 0, s);
        case 9: return launch_inv_segs<Tin, A, Tout, 9>(segs, nblocks, nullptr, 0, s);
        case 10: return launch_inv_segs<Tin, A, Tout, 10>(segs, nblocks, nullptr, 0, s);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_ifft_trunc_levels<double, double, double>(int, const InvLevel<double, double>*, int,
                                                                      hipStream_t);
template hipError_t launch_ifft_trunc_levels<float, ff32, ff32>(int, const InvLevel<float, ff32>*, int, hipStream_t);
template hipError_t launch_ifft_trunc_levels<float, double, ff32>(int, const InvLevel<float, ff32>*, int,
                                                                   hipStream_t);

template hipError_t launch_pad_fft<double>(int, const double*, cplx<double>*, int64_t, hipStream_t, int, int64_t,
                                           void*);
template hipError_t launch_pad_fft<float>(int, const float*, cplx<float>*, int64_t, hipStream_t, int, int64_t,
                                          void*);
template hipError_t launch_ifft_trunc<double, double, double>(int, const cplx<double>*, double*, int64_t,
                                                               hipStream_t, int, const int32_t*, void*, int);
template hipError_t launch_ifft_trunc<float, float, float>(int, const cplx<float>*, float*, int64_t, hipStream_t,
                                                             int, const int32_t*, void*, int);
template hipError_t launch_ifft_trunc<float, ff32, ff32>(int, const cplx<float>*, ff32*, int64_t, hipStream_t, int,
                                                         const int32_t*, void*, int);
template hipError_t launch_ifft_trunc<float, float, ff32>(int, const cplx<float>*, ff32*, int64_t, hipStream_t, int,
                                                          const int32_t*, void*, int);
template hipError_t launch_ifft_trunc<float, double, ff32>(int, const cplx<float>*, ff32*, int64_t, hipStream_t, int,
                                                           const int32_t*, void*, int);

}  // namespace lgfdev
