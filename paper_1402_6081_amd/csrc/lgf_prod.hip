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
#include <algorithm>
#include <cstdlib>

#include <type_traits>

#include "lgf_internal.h"

namespace lgfdev {

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Both
// blocked kernels map a 1D grid so that XCD x processes whole frequency chunks
// {c : c % 8 == x}, walking every group of such a chunk back to back: all reuse of a source
// spectrum within a chunk then stays in one L2.  Returns false for padding workgroups.
constexpr int kXcds = 8;
__device__ __forceinline__ bool xcd_tile_at(int L, int nchunks, int ngroupblocks, int& chunk, int& gblock) {
    const int xcd = L % kXcds, k = L / kXcds;
    chunk = (k / ngroupblocks) * kXcds + xcd;
    gblock = k % ngroupblocks;
    return chunk < nchunks;
}
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

// Keeps the compiler from moving instructions across this point.  Placed after a batch of
// independent gathers, it keeps them issued together (all in flight at once) instead of
// each load being sunk to its first use, which left one or two loads in flight per wave.
__device__ __forceinline__ void issue_fence() { __builtin_amdgcn_sched_barrier(0); }

// Coefficient lane_off of item `item` in a frequency chunk whose items start at the
// wave-uniform `base` (64 coefficients per item).  A 32-bit byte offset from a uniform base
// lets the gather use a scalar base register plus one vector offset instead of 64-bit
// address arithmetic per load (the launchers check that a chunk spans less than 4 GiB).
template <typename T>
__device__ __forceinline__ cplx<T> load_item(const cplx<T>* base, int item, int lane_off) {
    const uint32_t off = ((uint32_t)item * 64u + (uint32_t)lane_off) * (uint32_t)sizeof(cplx<T>);
    return *reinterpret_cast<const cplx<T>*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__host__ __forceinline__ bool chunk_fits_u32(int64_t items) {
    return items * 64 * (int64_t)sizeof(cplx<T>) <= (int64_t)UINT32_MAX;
}

// ------------------------------------------------------------------ level 0
// Groups g: tgt8[g][c] = block 2J + c (c = cx | cy<<1 | cz<<2) or -1;
// src64[g][s] = source block 2J + (sx-1, sy-1, sz-1), s = sx + 4 sy + 16 sz, or the zero
// sentinel item (index nsrc) when that block is not a source.  fhat holds nsrc + 1 items
// (the last is 0), uhat ntgt items (targets and sources are numbered separately, so the
// evaluation blocks may differ from the source blocks).
// A lane owns FPL consecutive frequencies: FPL = 1, a wave covers one 64-frequency chunk;
// FPL = 2 (FP32), a wave covers two consecutive chunks, lanes 0-31 the first and 32-63 the
// second, each lane loading 16 bytes per item as the FP64 lanes do.  The waves of a
// workgroup are different groups of the same chunk(s) and share the kernel tile in LDS: the
// 27 near offsets, row (dx+1) + 3 (dy+1) + 9 (dz+1).  A workgroup serves `rounds` blocks of
// groups in turn with that tile.  Every frequency is computed with the
// same arithmetic in the same order whatever FPL and the number of waves.
template <typename T, int FPL>
struct alignas(FPL * sizeof(cplx<T>)) LaneCoef {
    cplx<T> v[FPL];
};

template <typename T, int kNearWaves, bool kPrefetch, int FPL>
__global__ void __launch_bounds__(64 * kNearWaves)
    k_prod_near_grouped(const cplx<T>* __restrict__ fhat, const cplx<T>* __restrict__ khat,
                        const int32_t* __restrict__ tgt8, const int32_t* __restrict__ src64,
                        cplx<T>* __restrict__ uhat, int S, int ngroups, int nsrc, int ntgt, const SpecSym sym,
                        int rounds) {
    using V = LaneCoef<T, FPL>;
    __shared__ V tile[27 * 64];
    const int lane = threadIdx.x & 63;
    const int nchunks = (S + 63) / 64;  // the last chunk may be partial (frequencies w >= S unused)
    // a workgroup serves `rounds` blocks of kNearWaves groups of one chunk (block gb, then
    // gb + gstride, ...) with one kernel tile
    const int gstride = ((ngroups + kNearWaves - 1) / kNearWaves + rounds - 1) / rounds;
    int unit, gb;
    if (!xcd_tile((nchunks + FPL - 1) / FPL, gstride, unit, gb)) return;
    // this thread's chunk and first frequency in it; with FPL = 2 the second half of the
    // wave may fall past the last chunk, and then reads the first half's chunk and stores
    // nothing
    auto lane_pos = [&](int ln, int& ch, int& wl) {
        const int half = FPL == 2 ? (ln >> 5) : 0;
        ch = unit * FPL + half;
        wl = FPL == 2 ? 2 * (ln & 31) : ln;
    };
    int my_chunk, wl;
    lane_pos(lane, my_chunk, wl);
    const bool live = my_chunk < nchunks;
    if (!live) my_chunk = unit * FPL;
    const int w = my_chunk * 64 + wl;  // first frequency of this lane (S is a multiple of 64)
    if (sym.info != nullptr) {
        // reduced spectra: each thread fills rows of its own frequencies (the loop steps by
        // whole waves), decoded once; the rows' descriptions first, then all the gathers
        constexpr int NT = 64 * kNearWaves, NR = (27 * 64 + NT - 1) / NT;
        Freq3 om[FPL];
#pragma unroll
        for (int q = 0; q < FPL; ++q) om[q] = freq_of(w + q, sym.M);
        uint32_t inf[NR];
        bool use[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = (int)threadIdx.x + k * NT;
            use[k] = i < 27 * 64;
            inf[k] = use[k] ? sym.info[i >> 6] : 0u;
        }
        V kv[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int q = 0; q < FPL; ++q)
                kv[k].v[q] = use[k] && w + q < S ? sym_coef(khat, inf[k], om[q], sym.ncls, sym.M) : cplx<T>{T(0), T(0)};
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = (int)threadIdx.x + k * NT;
            if (i < 27 * 64) tile[i] = kv[k];
        }
    } else {
        for (int i = threadIdx.x; i < 27 * 64; i += 64 * kNearWaves) {
            int ch, wi;
            lane_pos(i & 63, ch, wi);
            if (ch >= nchunks) ch = unit * FPL;
            const int wt = ch * 64 + wi;
            tile[i] = wt < S ? *reinterpret_cast<const V*>(khat + spec_at(i >> 6, wt, 27)) : V{};
        }
    }
    __syncthreads();
    T ar[FPL][8], ai[FPL][8];
    const int32_t* sg = src64;  // this round's group: its 64 source items
    // the first chunk's items (wave-uniform base) and this lane's offset from it, in
    // coefficients: its chunk, then its frequencies within the item
    const cplx<T>* fbase = fhat + (int64_t)(unit * FPL) * (nsrc + 1) * 64;
    const uint32_t loff = ((uint32_t)(my_chunk - unit * FPL) * (uint32_t)(nsrc + 1) * 64u + (uint32_t)wl) *
                          (uint32_t)sizeof(cplx<T>);
    auto load = [&](int item) -> V {
        const uint32_t off = (uint32_t)item * 64u * (uint32_t)sizeof(cplx<T>) + loff;
        return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(fbase) + off);
    };
    // source z slab sz contributes to target slab cz through kernel rows dz = cz - (sz - 1).
    // Each of the slab's 18 kernel values (9 (dx, dy) x 2 target slabs) is read from LDS once
    // and applied to the 4 targets (cx, cy) whose source cx - dx, cy - dy lies in the slab.
    // (dy, dx) run from +1 down to -1, so every target still adds its sources in increasing
    // (sy, sx) order: the same terms in the same order as a loop over the sources.  The end
    // slabs reach one target slab only (sz = 0: cz = 0; sz = 3: cz = 1): the other row would
    // be |dz| = 2, outside the near field.  The end slabs are unrolled out of the slab loop
    // with that row dropped at compile time (measured: the 256^3 FP64 Prod 698 -> 677 us,
    // FP32 371 -> 364 us, against one wave-uniform branch per row).
    // END: 0 for the first slab, 3 for the last, -1 for a middle one, so the end slabs'
    // skipped row is a compile-time choice and no slab body has a branch
    auto slab = [&](auto endc, int sz, const V(&f)[16]) {
        constexpr int END = decltype(endc)::value;
        // kernel row bases for cz = 0 (dz = 1 - sz) and cz = 1 (dz = 2 - sz); an end slab's
        // unused one is pointed at row 0
        const V* t0 = tile + 9 * (sz < 3 ? 2 - sz : 0) * 64 + lane;
        const V* t1 = tile + 9 * (sz > 0 ? 3 - sz : 0) * 64 + lane;
#pragma unroll
        for (int dy = 1; dy >= -1; --dy) {
#pragma unroll
            for (int dx = 1; dx >= -1; --dx) {
#pragma unroll
                for (int cz = 0; cz < 2; ++cz) {
                    if (cz ? END == 0 : END == 3) continue;  // |dz| = 2 (compile-time)
                    const V k = (cz ? t1 : t0)[((dx + 1) + 3 * (dy + 1)) * 64];
#pragma unroll
                    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
                        for (int cx = 0; cx < 2; ++cx) {
                            const int c = cx | (cy << 1) | (cz << 2);
                            const int sxy = (cx - dx + 1) + 4 * (cy - dy + 1);
#pragma unroll
                            for (int q = 0; q < FPL; ++q) cmac(ar[q][c], ai[q][c], f[sxy].v[q], k.v[q]);
                        }
                }
            }
        }
    };
    // the half h of slab sz: source rows sy = 2h + j (j = 0, 1) in f[4 j + sx]; a target
    // row cy meets them through dy = cy - sy + 1, so half 0 uses dy = 1, 0 and half 1
    // dy = 0, -1
    auto half = [&](auto endc, int sz, auto hc, const V(&f)[8]) {
        constexpr int END = decltype(endc)::value, h = decltype(hc)::value;
        const V* t0 = tile + 9 * (sz < 3 ? 2 - sz : 0) * 64 + lane;
        const V* t1 = tile + 9 * (sz > 0 ? 3 - sz : 0) * 64 + lane;
#pragma unroll
        for (int dy = 1; dy >= -1; --dy) {
#pragma unroll
            for (int dx = 1; dx >= -1; --dx) {
#pragma unroll
                for (int cz = 0; cz < 2; ++cz) {
                    if (cz ? END == 0 : END == 3) continue;  // |dz| = 2 (compile-time)
                    if (h == 0 ? dy < 0 : dy > 0) continue;  // no target row meets this half
                    const V k = (cz ? t1 : t0)[((dx + 1) + 3 * (dy + 1)) * 64];
#pragma unroll
                    for (int cy = 0; cy < 2; ++cy) {
                        const int sy = cy - dy + 1;
                        if (sy < 2 * h || sy > 2 * h + 1) continue;
#pragma unroll
                        for (int cx = 0; cx < 2; ++cx) {
                            const int c = cx | (cy << 1) | (cz << 2);
                            const int sxy = (cx - dx + 1) + 4 * (sy - 2 * h);
#pragma unroll
                            for (int q = 0; q < FPL; ++q) cmac(ar[q][c], ai[q][c], f[sxy].v[q], k.v[q]);
                        }
                    }
                }
            }
        }
    };
    using First = std::integral_constant<int, 0>;
    using Mid = std::integral_constant<int, -1>;
    using Last = std::integral_constant<int, 3>;
    using H0 = std::integral_constant<int, 0>;
    using H1 = std::integral_constant<int, 1>;
#pragma unroll 1
    for (int r = 0; r < rounds; ++r) {
        const int g = wave_uniform((gb + r * gstride) * kNearWaves + (threadIdx.x >> 6));
        if (g >= ngroups) break;
        // 4-wave workgroups whose groups all exist step through the source slabs together
        // (a barrier before each slab's, or half slab's, loads): the waves' groups are
        // neighbours and share half their sources, which the lockstep serves from L1 (the
        // 256^3 Prod 689 -> 662 us FP64, 363 -> 353 us FP32; with 8 waves it was slower).
        // The condition is uniform over the workgroup, so every wave meets the same barriers.
        const bool lockstep = kNearWaves == 4 && (gb + r * gstride) * kNearWaves + kNearWaves <= ngroups;
#pragma unroll
        for (int q = 0; q < FPL; ++q)
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                ar[q][c] = T(0);
                ai[q][c] = T(0);
            }
        sg = src64 + (int64_t)g * 64;
        if constexpr (kPrefetch) {
            // half slabs (source rows sy = 2h, 2h + 1) through two buffers of 8 values: the next
            // half's loads are in flight while this half is consumed, in the registers the
            // one-slab form uses for its 16 values.  A target meets the rows of the first half
            // before those of the second, so it adds the same terms in the same order.
            V fa[8], fb[8];
            auto ld = [&](int sz, int h, V(&x)[8]) {
                if (lockstep) __syncthreads();
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = load(sg[sz * 16 + 8 * h + i]);
            };
            ld(0, 0, fa);
            ld(0, 1, fb);
            issue_fence();
            half(First{}, 0, H0{}, fa);
            ld(1, 0, fa);
            issue_fence();
            half(First{}, 0, H1{}, fb);
#pragma unroll 1
            for (int sz = 1; sz < 3; ++sz) {
                ld(sz, 1, fb);
                issue_fence();
                half(Mid{}, sz, H0{}, fa);
                ld(sz + 1, 0, fa);
                issue_fence();
                half(Mid{}, sz, H1{}, fb);
            }
            ld(3, 1, fb);
            issue_fence();
            half(Last{}, 3, H0{}, fa);
            issue_fence();
            half(Last{}, 3, H1{}, fb);
        } else {
            V f[16];
            if (lockstep) __syncthreads();
#pragma unroll
            for (int sxy = 0; sxy < 16; ++sxy) f[sxy] = load(sg[sxy]);
            issue_fence();
            slab(First{}, 0, f);
#pragma unroll 1
            for (int sz = 1; sz < 3; ++sz) {  // the middle source z slabs; x and y unrolled
                if (lockstep) __syncthreads();
#pragma unroll
                for (int sxy = 0; sxy < 16; ++sxy) f[sxy] = load(sg[sz * 16 + sxy]);
                issue_fence();
                slab(Mid{}, sz, f);
            }
            if (lockstep) __syncthreads();
#pragma unroll
            for (int sxy = 0; sxy < 16; ++sxy) f[sxy] = load(sg[48 + sxy]);
            issue_fence();
            slab(Last{}, 3, f);
        }
        if (!live || w >= S) continue;  // (S is even, so a lane's two frequencies are both below it or not)
        const int32_t* tg = tgt8 + (int64_t)g * 8;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int t = tg[c];
            if (t >= 0) {
                // streamed past the caches: the output is read once, by the inverse transform, and
                // must not evict the source spectra this kernel re-reads (measured: this Prod 15%
                // faster, the inverse 10% slower, the pair 7% faster at 128^3 FP64)
                typedef T vec_t __attribute__((ext_vector_type(2 * FPL)));  // one store per lane
                vec_t o;
#pragma unroll
                for (int q = 0; q < FPL; ++q) {
                    o[2 * q] = ar[q][c];
                    o[2 * q + 1] = ai[q][c];
                }
                __builtin_nontemporal_store(o, reinterpret_cast<vec_t*>(uhat + spec_at(t, w, ntgt)));
            }
        }
    }
}

// ------------------------------------------------------------------ levels >= 1, sibling blocked
// Parents J (level l+1): src216[J][e * 8 + cs] = level-l interval 2(J + e') + cs with
// e' = (ex-1, ey-1, ez-1), e = ex + 3 ey + 9 ez, or the zero sentinel item (index nitems);
// child8[J][c] = target 2J + c (or -1).  khat: 343 offsets, id (Dx+3) + 7 (Dy+3) + 49 (Dz+3).
//
// The target child c receives source child cs of neighbour e at offset D = c - cs - 2e'.
// Register blocking: a lane owns one frequency of one parent and accumulates CPL of its 8
// children (the subset Q of the children is fixed per wave, so all its index arithmetic is
// compile-time).  Per neighbour e the lane loads the 8 source coefficients once; its
// (child, source child) pairs need only the kernel values at delta = c - cs, each read once
// from LDS and applied to every pair with that delta.  The delta loop is unrolled and has
// no branch: the interaction-list condition |D|_inf >= 2 is met by zero kernel rows at the
// near offsets (the centre neighbour, all of whose pairs are near, is skipped whole).
// Every child sums its terms in the same order (neighbour e, then delta) whatever CPL and
// the number of waves, so all variants give identical results.  A neighbour whose children
// are all the zero sentinel for every parent of a wave (absent intervals, or intervals
// without sources) is skipped by that wave: the terms it would add are exact zeros.
// Lanes: F consecutive frequencies (one 128-byte segment of a spectrum) x 64/F parents.
// The workgroup's waves share the [343][F] kernel tile (its Dz >= 0 half, below) and the
// parents' source indices in LDS.
template <typename T>
struct M2LShape {
    static constexpr int F = 128 / (int)sizeof(cplx<T>);  // frequencies per chunk: 8 FP64, 16 FP32
    static constexpr int PPW = 64 / F;                     // parents per wave
};
// The kernel tile keeps the half with Dz >= 0 (196 of its 343 rows): FP64 25 instead of
// 44 KB of LDS, so four 4-wave workgroups share a CU (FP32 five).  The kernel spectra of opposite
// offsets are complex conjugates (the kernel is real and even, Sec. 2.1, and its padded
// tile is placed symmetrically about the origin: offset r at circulant index r mod M, zero
// at M/2; so the -D tile is the D tile reflected, and its DFT the conjugate).  An offset
// with Dz < 0 is read as the conjugate of the row of -D.  In a neighbour step the deltas of
// one dz slab share Dz = dz - 2 ez, so a slab either reads D or conjugates throughout.
template <typename T>
struct M2LTile {
    static constexpr bool kHalf = true;  // (the full tile: kRow0 = 0, every slab reads D)
    static constexpr int kRow0 = kHalf ? 147 : 0;  // first row id kept: D = (-3, -3, 0)
    static constexpr int kRows = 343 - kRow0;
};

// v with its sign flipped when flip (wave-uniform): one integer XOR on the sign bit
template <typename T>
__device__ __forceinline__ T neg_if(T v, bool flip) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long m = (unsigned long long)flip << 63;
        return __longlong_as_double(__double_as_longlong(v) ^ (long long)m);
    } else {
        const unsigned m = (unsigned)flip << 31;
        return __uint_as_float(__float_as_uint(v) ^ m);
    }
}

// ar + i ai += f * conj(k): the conjugate's sign goes into the FMAs' operands (the same
// roundings as cmac with the sign-flipped k)
template <typename T>
__device__ __forceinline__ void cmac_conj(T& ar, T& ai, const cplx<T>& f, const cplx<T>& k) {
    ar = fma(f.x, k.x, ar);
    ar = fma(f.y, k.y, ar);
    ai = fma(-f.x, k.y, ai);
    ai = fma(f.y, k.x, ai);
}

// child i of subset Q when a lane accumulates CPL children (subsets split z, then y, then x)
template <int CPL, int Q>
__device__ constexpr int m2l_child(int i) { return Q * CPL + i; }

// The deltas of one dz slab applied to this lane's children.  kb points at the row of
// delta d = 0; delta d reads kb[s (dx + 7 dy) F] with s = 1, or s = -1 when the slab reads
// the rows of -D.  CONJ: 0 reads D, 1 conjugates (compile-time), 2 decides by flip
// (wave-uniform, one sign-bit XOR per kernel value).  (ex, ey, ez) is the neighbour's
// offset e': a delta whose offset D = d - 2e' is near (|D|_inf <= 1, a zero row of the
// tile) adds nothing and is skipped; with e' known at compile time, as in the unrolled
// neighbour loops, that costs no instruction.
template <typename T, int CPL, int Q, int CONJ>
__device__ __forceinline__ void m2l_slab(int dz, const cplx<T>* kb, bool flip, const cplx<T> (&fa)[8],
                                         T (&ar)[CPL], T (&ai)[CPL], int ex, int ey, int ez) {
    constexpr int F = M2LShape<T>::F;
#pragma unroll
    for (int dd = 0; dd < 9; ++dd) {
        const int dx = dd % 3 - 1, dy = dd / 3 - 1;
        const int Dx = dx - 2 * ex, Dy = dy - 2 * ey, Dz = dz - 2 * ez;
        if (Dx >= -1 && Dx <= 1 && Dy >= -1 && Dy <= 1 && Dz >= -1 && Dz <= 1) continue;  // near
        bool used = false;  // compile-time: does a child of this subset pair with delta d?
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
            const int c = m2l_child<CPL, Q>(i);
            const int csx = (c & 1) - dx, csy = ((c >> 1) & 1) - dy, csz = (c >> 2) - dz;
            used |= csx >= 0 && csx <= 1 && csy >= 0 && csy <= 1 && csz >= 0 && csz <= 1;
        }
        if (!used) continue;
        cplx<T> k;
        if constexpr (CONJ == 2) {
            k = kb[(flip ? -(dx + 7 * dy) : dx + 7 * dy) * F];
            k.y = neg_if<T>(k.y, flip);
        } else {
            k = kb[(CONJ ? -(dx + 7 * dy) : dx + 7 * dy) * F];
        }
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
            const int c = m2l_child<CPL, Q>(i);
            const int csx = (c & 1) - dx, csy = ((c >> 1) & 1) - dy, csz = (c >> 2) - dz;
            if (csx < 0 || csx > 1 || csy < 0 || csy > 1 || csz < 0 || csz > 1) continue;  // compile-time
            if constexpr (CONJ == 1)
                cmac_conj(ar[i], ai[i], fa[csx | (csy << 1) | (csz << 2)], k);
            else
                cmac(ar[i], ai[i], fa[csx | (csy << 1) | (csz << 2)], k);
        }
    }
}

// The contribution of neighbour e to this lane's children, with source values fa.  The
// kernel tile holds zeros in the near-offset rows (|D| <= 1), which only near pairs would
// read; the slabs skip those deltas (exact zero terms: the sums' bits are the same either
// way).  The deltas of one dz slab form one scheduling region, so the multiply-adds of
// several deltas interleave.  LAYER = ez of the neighbours this code serves when known at
// compile time (each slab then reads D or conjugates in code of its own), else 2.
template <typename T, int CPL, int Q, int LAYER = 2>
__device__ __forceinline__ void m2l_neighbour(int e, const cplx<T> (&fa)[8], const cplx<T>* tk, T (&ar)[CPL],
                                              T (&ai)[CPL]) {
    constexpr int F = M2LShape<T>::F;
    const int ex = e % 3 - 1, ey = (e / 3) % 3 - 1, ez = LAYER == 2 ? e / 9 - 1 : LAYER;  // wave-uniform
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        if constexpr (M2LTile<T>::kHalf) {
            // the halved tile's row (Dx+3) + 7 (Dy+3) + 49 Dz holds D, Dz = dz - 2 ez
            const cplx<T>* plain = tk + ((3 - 2 * ex) + 7 * (3 - 2 * ey) + 49 * (dz - 2 * ez)) * F;
            const cplx<T>* mirror = tk + ((3 + 2 * ex) + 7 * (3 + 2 * ey) + 49 * (2 * ez - dz)) * F;
            if constexpr (LAYER == 2) {
                const bool flip = dz - 2 * ez < 0;
                m2l_slab<T, CPL, Q, 2>(dz, flip ? mirror : plain, flip, fa, ar, ai, ex, ey, ez);
            } else if constexpr (LAYER < 0) {
                m2l_slab<T, CPL, Q, 0>(dz, plain, false, fa, ar, ai, ex, ey, ez);
            } else {
                // LAYER = 1: every slab conjugates; LAYER = 0: the dz = -1 slab only
                if (LAYER == 1 || dz < 0)
                    m2l_slab<T, CPL, Q, 1>(dz, mirror, true, fa, ar, ai, ex, ey, ez);
                else
                    m2l_slab<T, CPL, Q, 0>(dz, plain, false, fa, ar, ai, ex, ey, ez);
            }
        } else {
            m2l_slab<T, CPL, Q, 0>(dz, tk + ((3 - 2 * ex) + 7 * (3 - 2 * ey) + 49 * (3 + dz - 2 * ez)) * F, false,
                                   fa, ar, ai, ex, ey, ez);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <typename T, typename IdxT>
__device__ __forceinline__ void m2l_load(int e, const cplx<T>* __restrict__ fb, int wl, const IdxT* si,
                                         cplx<T> (&f)[8]) {
    const int ee = e < 27 ? e : 26;  // past the end: a harmless reload of the last neighbour
#pragma unroll
    for (int cs = 0; cs < 8; ++cs) f[cs] = load_item(fb, (int)si[ee * 8 + cs], wl);
}

// Neighbours in order e = 0..26 through a pipeline of source buffers: with three, the
// sources of e+1 and e+2 are in flight while e is consumed.
// live: wave-uniform mask, bit e set when neighbour e holds a source for some parent of
// the wave.
template <typename T, int CPL, int Q, typename IdxT>
__device__ __forceinline__ void m2l_lane(const cplx<T>* __restrict__ fb, int wl, const IdxT* si,
                                         const cplx<T>* tk, uint32_t live, T (&ar)[CPL], T (&ai)[CPL]) {
    if constexpr (CPL >= 4) {
        // 4 or 8 children per lane: two buffers, the next neighbour's sources in flight
        // while one is consumed.  The FP64 four-children lane then needs 90 registers
        // instead of 164 (9-12% faster on the larger levels); the all-children lane 116
        // instead of 152, and with the halved kernel tile four 4-wave workgroups share a CU
        // (with the conjugation compiled per layer, below: the 256^3 M2L 550 -> 432 us, the
        // 128^3 one 97 -> 81 us, the Table 2 scheme cubes 11-12% faster than with the full
        // tile).  FP32 with the unrolled layers: 74 instead of 92 registers, six waves per
        // SIMD instead of five, the 256^3 M2L 252 -> 234 us.  The one- and two-children
        // lanes keep three buffers, which measured faster for them.
        // one loop per layer ez of neighbours (9 each), so that every slab's conjugation is
        // known at compile time; the buffer holding the next neighbour alternates between
        // layers (9 is odd).  The loops are unrolled: each neighbour's offset is then a
        // constant and its near deltas drop out of the code (the 256^3 M2L 435 -> 400 us
        // FP64, 273 -> 245 us FP32; the n_I = 17 scheme's 416 -> 394 us, same bits)
        cplx<T> fa[8], fbuf[8];
        auto layer = [&](auto lc, int e0, cplx<T>(&x)[8], cplx<T>(&y)[8]) {
            constexpr int LY = decltype(lc)::value;
#pragma unroll
            for (int e = e0; e < e0 + 9; e += 2) {
                m2l_load<T, IdxT>(e + 1, fb, wl, si, y);
                issue_fence();
                if (live & (1u << e)) m2l_neighbour<T, CPL, Q, LY>(e, x, tk, ar, ai);
                if (e + 1 < e0 + 9) {
                    m2l_load<T, IdxT>(e + 2, fb, wl, si, x);
                    issue_fence();
                    if (live & (2u << e)) m2l_neighbour<T, CPL, Q, LY>(e + 1, y, tk, ar, ai);
                }
            }
        };
        m2l_load<T, IdxT>(0, fb, wl, si, fa);
        layer(std::integral_constant<int, -1>{}, 0, fa, fbuf);  // leaves neighbour 9 in fbuf
        layer(std::integral_constant<int, 0>{}, 9, fbuf, fa);   // leaves neighbour 18 in fa
        layer(std::integral_constant<int, 1>{}, 18, fa, fbuf);
    } else {
        cplx<T> fa[8], fbuf[8], fc[8];
        m2l_load<T, IdxT>(0, fb, wl, si, fa);
        m2l_load<T, IdxT>(1, fb, wl, si, fbuf);
        // one loop per layer ez (9 neighbours, three per iteration, so the buffers line up),
        // so that every slab's conjugation is known at compile time (the halved tile: the
        // 256^3 FP32 M2L 282 -> 266 us, the n_I = 17 scheme's 340 -> 267 us)
        auto layer = [&](auto lc, int e0) {
            constexpr int LY = decltype(lc)::value;
#pragma unroll
            for (int e = e0; e < e0 + 9; e += 3) {
                m2l_load<T, IdxT>(e + 2, fb, wl, si, fc);
                issue_fence();
                if (live & (1u << e)) m2l_neighbour<T, CPL, Q, LY>(e, fa, tk, ar, ai);
                m2l_load<T, IdxT>(e + 3, fb, wl, si, fa);
                issue_fence();
                if (live & (2u << e)) m2l_neighbour<T, CPL, Q, LY>(e + 1, fbuf, tk, ar, ai);
                m2l_load<T, IdxT>(e + 4, fb, wl, si, fbuf);
                issue_fence();
                if (live & (4u << e)) m2l_neighbour<T, CPL, Q, LY>(e + 2, fc, tk, ar, ai);
            }
        };
        layer(std::integral_constant<int, -1>{}, 0);
        layer(std::integral_constant<int, 0>{}, 9);
        layer(std::integral_constant<int, 1>{}, 18);
    }
}

template <typename T, int CPL, int Q = 0, typename IdxT>
__device__ __forceinline__ void m2l_dispatch(int q, const cplx<T>* fb, int wl, const IdxT* si,
                                             const cplx<T>* tk, uint32_t live, T (&ar)[CPL], T (&ai)[CPL]) {
    if constexpr (Q + 1 < 8 / CPL) {
        if (q != Q) {
            m2l_dispatch<T, CPL, Q + 1, IdxT>(q, fb, wl, si, tk, live, ar, ai);
            return;
        }
    }
    m2l_lane<T, CPL, Q, IdxT>(fb, wl, si, tk, live, ar, ai);
}

// One launch may cover several levels (segments of the grid, each with its own spectra,
// lists, kernel spectra and spectrum size S): the coarse levels' small
// M2L then runs inside the level-1 launch instead of as latency-bound launches of its own.
// Segment k owns the workgroups [start_k, start_{k+1}); each start is a multiple of the
// XCD count, so every segment keeps the XCD-aware chunk mapping.
template <typename T>
struct FarSeg {
    const cplx<T>* fhat;
    const cplx<T>* khat;
    const int32_t* child8;
    const int32_t* src216;
    cplx<T>* uhat;
    int nparents, nitems, nsrc, ngroupblocks, start, S;
    SpecSym sym;  // reduced kernel spectra (sym.info == nullptr: one spectrum per offset)
};
template <typename T>
struct FarSegs {
    FarSeg<T> s[kMaxFarSegs];
    int n;
};

// tile row r = (Dx+3) + 7 (Dy+3) + 49 (Dz+3) of a near offset (|D| <= 1 on every axis)
__device__ __forceinline__ bool m2l_near_row(int r) {
    const int dx = r % 7 - 3, dy = (r / 7) % 7 - 3, dz = r / 49 - 3;
    return dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
}

template <typename T, int kFarWaves, int CPL, typename IdxT>
__global__ void __launch_bounds__(64 * kFarWaves * (8 / CPL))
    k_prod_far_sib(const FarSegs<T> segs) {
    constexpr int F = M2LShape<T>::F;
    constexpr int PPW = M2LShape<T>::PPW;
    constexpr int NQ = 8 / CPL;             // waves per group of parents (one per child subset)
    constexpr int PPG = PPW * kFarWaves;    // parents per workgroup
    constexpr int NT = 64 * kFarWaves * NQ;
    constexpr int kRows = M2LTile<T>::kRows, kRow0 = M2LTile<T>::kRow0;
    __shared__ cplx<T> tile[kRows * F];
    __shared__ IdxT sidx[PPG * 216];  // 16-bit when every level's items fit (less LDS)
    __shared__ uint32_t live[kFarWaves];  // per group of PPW parents: neighbours holding a source
    // this workgroup's segment (uniform selects over the kernel arguments)
    FarSeg<T> g = segs.s[0];
#pragma unroll
    for (int k = 1; k < kMaxFarSegs; ++k)
        if (k < segs.n && (int)blockIdx.x >= segs.s[k].start) g = segs.s[k];
    const cplx<T>* __restrict__ fhat = g.fhat;
    const cplx<T>* __restrict__ khat = g.khat;
    const int32_t* __restrict__ child8 = g.child8;
    const int32_t* __restrict__ src216 = g.src216;
    cplx<T>* __restrict__ uhat = g.uhat;
    const int nparents = g.nparents, nitems = g.nitems, nsrc = g.nsrc, S = g.S;
    const int nchunks = (S + F - 1) / F;
    int chunk, pb;
    if (!xcd_tile_at((int)blockIdx.x - g.start, nchunks, g.ngroupblocks, chunk, pb)) return;
    const int w0 = chunk * F;
    // reduced spectra: NT is a multiple of F, so every row a thread fills has the same
    // frequency, decoded once
    if (g.sym.info != nullptr) {
        // every row's description first, then all the (dependent) gathers, so the loads of
        // a thread's rows are in flight together
        constexpr int NR = (kRows * F + NT - 1) / NT;
        const int jj = (int)threadIdx.x % F;
        const bool wok = w0 + jj < S;
        const Freq3 om = wok ? freq_of(w0 + jj, g.sym.M) : Freq3{};
        uint32_t inf[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = (int)threadIdx.x + k * NT;
            inf[k] = i < kRows * F ? g.sym.info[kRow0 + i / F] : 0u;
        }
        cplx<T> kv[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = (int)threadIdx.x + k * NT;
            kv[k] = (i < kRows * F && wok && !m2l_near_row(kRow0 + i / F))
                        ? sym_coef(khat, inf[k], om, g.sym.ncls, g.sym.M)
                        : cplx<T>{T(0), T(0)};
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = (int)threadIdx.x + k * NT;
            if (i < kRows * F) tile[i] = kv[k];
        }
    } else {
        for (int i = threadIdx.x; i < kRows * F; i += NT) {
            const int r = kRow0 + i / F, jj = i % F;
            tile[i] = (w0 + jj < S && !m2l_near_row(r)) ? khat[spec_at(r, w0 + jj, 343)] : cplx<T>{T(0), T(0)};
        }
    }
    for (int i = threadIdx.x; i < PPG * 216; i += NT) {
        const int Jl = i / 216, k = i - Jl * 216;
        const int J = pb * PPG + Jl;
        sidx[i] = (IdxT)(J < nparents ? src216[(int64_t)J * 216 + k] : nsrc);  // padding parents read zeros
    }
    if (threadIdx.x < kFarWaves) live[threadIdx.x] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < kFarWaves * 27; i += NT) {
        const int g = i / 27, e = i - g * 27;
        bool any = false;
        for (int jl = g * PPW; jl < (g + 1) * PPW; ++jl)
#pragma unroll
            for (int cs = 0; cs < 8; ++cs) any |= (int)sidx[jl * 216 + e * 8 + cs] != nsrc;
        if (any) atomicOr(&live[g], 1u << e);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int q = wave % NQ, pw = wave / NQ;
    const int j = lane % F;
    const int Jl = pw * PPW + lane / F;
    const int J = pb * PPG + Jl;
    const int w = w0 + j;  // may exceed S in the last chunk: computed, never stored
    const cplx<T>* fb = fhat + (int64_t)(w0 >> 6) * (nsrc + 1) * 64;  // this chunk's items (uniform)
    T ar[CPL], ai[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
        ar[i] = T(0);
        ai[i] = T(0);
    }
    // the centre neighbour (the parent itself) holds only near pairs
    m2l_dispatch<T, CPL, 0, IdxT>(q, fb, w & 63, sidx + Jl * 216, tile + j,
                                  (uint32_t)wave_uniform((int)live[pw]) & ~(1u << 13), ar, ai);
    if (J >= nparents || w >= S) return;
    const int32_t* c8 = child8 + (int64_t)J * 8 + q * CPL;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
        const int t = c8[i];
        if (t >= 0) uhat[spec_at(t, w, nitems)] = cplx<T>{ar[i], ai[i]};
    }
}

// ------------------------------------------------------------------ generic CSR (top level)
constexpr int kProdThreads = 256;

// Targets tgt[i] (i = blockIdx.x) with list entries [ptr[i], ptr[i+1]).
template <typename T>
__global__ void __launch_bounds__(kProdThreads)
    k_prod_far(const cplx<T>* __restrict__ fhat, const cplx<T>* __restrict__ khat,
               const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
               const int32_t* __restrict__ off, const int32_t* __restrict__ tgt, cplx<T>* __restrict__ uhat, int S,
               int nitems, int noff, int nsrc, const SpecSym sym) {
    const int w = blockIdx.y * kProdThreads + threadIdx.x;
    const int64_t i = blockIdx.x;
    if (w >= S) return;
    const bool red = sym.info != nullptr;
    Freq3 om{};
    if (red) om = freq_of(w, sym.M);
    const int64_t P = tgt[i];
    const int e0 = ptr[i], e1 = ptr[i + 1];
    T ar = T(0), ai = T(0);
    for (int e = e0; e < e1; ++e) {
        const int q = src[e];
        const int o = off[e];
        const cplx<T> f = fhat[spec_at(q, w, nsrc + 1)];
        const cplx<T> k = red ? sym_coef(khat, sym.info[o], om, sym.ncls, sym.M) : khat[spec_at(o, w, noff)];
        cmac(ar, ai, f, k);
    }
    uhat[spec_at(P, w, nitems)] = cplx<T>{ar, ai};
}

// Frequencies per lane of the level-0 Prod: 2 in FP32, so that every lane moves 16 bytes
// per item as in FP64 (half the load and store instructions per byte).
template <typename T>
constexpr int kNearFpl = sizeof(T) == 4 ? 2 : 1;

// Group blocks per workgroup of the level-0 Prod: every round reuses the workgroup's kernel
// tile, and the smaller grid leaves CUs to the far-field kernels running beside it (graph
// solves, 4-wave workgroups: 256^3 FP32 0.947 -> 0.929 ms with 2 rounds, 128^3 FP64
// 0.277 -> 0.259 ms and FP32 0.154 -> 0.149 ms with 4; the same bits)
static int near_rounds(int nunits, int nblocks) {
    const int64_t wgs = (int64_t)nunits * nblocks;
    return wgs >= 16384 ? 2 : (wgs >= 1024 ? 4 : 1);
}

template <typename T, int NW, bool PF>
static hipError_t near_nw(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* tgt8, const int32_t* src64,
                          cplx<T>* uhat, int64_t ngroups, int64_t nsrc, int64_t ntgt, int S, hipStream_t s,
                          const SpecSym& sym) {
    constexpr int FPL = kNearFpl<T>;
    const int nunits = ((S + 63) / 64 + FPL - 1) / FPL, nblocks = (int)((ngroups + NW - 1) / NW);
    const int rounds = near_rounds(nunits, nblocks);
    const unsigned grid = xcd_grid(nunits, (nblocks + rounds - 1) / rounds);
    return lgf_launch(k_prod_near_grouped<T, NW, PF, FPL>, dim3(grid), dim3(64 * NW), 0, s, fhat, khat, tgt8,
                      src64, uhat, S, (int)ngroups, (int)nsrc, (int)ntgt, sym, rounds);
}

template <typename T, bool PF>
static hipError_t near_pf(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* tgt8, const int32_t* src64,
                          cplx<T>* uhat, int64_t ngroups, int64_t nsrc, int64_t ntgt, int S, int waves,
                          hipStream_t s, const SpecSym& sym) {
    switch (waves) {
        case 2: return near_nw<T, 2, PF>(fhat, khat, tgt8, src64, uhat, ngroups, nsrc, ntgt, S, s, sym);
        case 8: return near_nw<T, 8, PF>(fhat, khat, tgt8, src64, uhat, ngroups, nsrc, ntgt, S, s, sym);
        default: return near_nw<T, 4, PF>(fhat, khat, tgt8, src64, uhat, ngroups, nsrc, ntgt, S, s, sym);
    }
}

template <typename T>
hipError_t launch_prod_near(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* tgt8, const int32_t* src64,
                            cplx<T>* uhat, int64_t ngroups, int64_t nsrc, int64_t ntgt, int S, int waves,
                            int prefetch, hipStream_t s, const SpecSym& sym) {
    if (ngroups <= 0) return hipSuccess;
    // a lane's 32-bit offsets span kNearFpl consecutive chunks of the source spectra
    if (S <= 0 || S % 2 || !chunk_fits_u32<T>((nsrc + 1) * kNearFpl<T>) || !sym_fits(sym, S))
        return hipErrorInvalidValue;
    return prefetch ? near_pf<T, true>(fhat, khat, tgt8, src64, uhat, ngroups, nsrc, ntgt, S, waves, s, sym)
                    : near_pf<T, false>(fhat, khat, tgt8, src64, uhat, ngroups, nsrc, ntgt, S, waves, s, sym);
}

// LGF_M2L_WIDE_LISTS=1 in the environment keeps the 32-bit list entries at every level
// size, the form levels of 65535 or more items take (read at each launch; the same bits
// either way).
static bool m2l_wide_lists() {
    const char* v = std::getenv("LGF_M2L_WIDE_LISTS");
    return v && v[0] == '1';
}

template <typename T, int NW, int CPL>
static hipError_t far_nw(const FarLevel<T>* lv, int nlev, hipStream_t s) {
    constexpr int F = M2LShape<T>::F, PPG = M2LShape<T>::PPW * NW;
    FarSegs<T> segs{};
    unsigned grid = 0;
    for (int k = 0; k < nlev; ++k) {
        const int ngb = (int)((lv[k].nparents + PPG - 1) / PPG);
        const int nchunks = (lv[k].S + F - 1) / F;
        segs.s[k] = FarSeg<T>{lv[k].fhat,      lv[k].khat,         lv[k].child8,       lv[k].src216,
                              lv[k].uhat,      (int)lv[k].nparents, (int)lv[k].nitems, (int)lv[k].nsrc,
                              ngb,             (int)grid,           lv[k].S,
                              lv[k].sym};
        grid += xcd_grid(nchunks, ngb);  // a multiple of the XCD count
    }
    segs.n = nlev;
    // 16-bit list entries in LDS when every level's items (and the sentinel) fit: less LDS
    // per workgroup, so more workgroups share a CU
    bool idx16 = !m2l_wide_lists();
    for (int k = 0; k < nlev; ++k) idx16 = idx16 && lv[k].nsrc < 65535;
    if (idx16)
        return lgf_launch(k_prod_far_sib<T, NW, CPL, uint16_t>, dim3(grid), dim3(64 * NW * (8 / CPL)), 0, s, segs);
    return lgf_launch(k_prod_far_sib<T, NW, CPL, int32_t>, dim3(grid), dim3(64 * NW * (8 / CPL)), 0, s, segs);
}

template <typename T, int CPL>
static hipError_t far_cpl(const FarLevel<T>* lv, int nlev, int waves, hipStream_t s) {
    // at most 16 waves (1024 threads) per workgroup, and at most 8 in FP64, whose pipeline
    // needs more than the 128 registers a lane gets in a 16-wave workgroup.  Larger groups
    // share one kernel tile among more parents (more waves per CU for the same LDS).
    constexpr int kMaxWaves = sizeof(T) == 8 ? 8 : 16;
    constexpr int kMaxGroups = kMaxWaves / (8 / CPL);
    const int g = waves < kMaxGroups ? waves : kMaxGroups;
    if constexpr (kMaxGroups >= 16)
        if (g >= 16) return far_nw<T, 16, CPL>(lv, nlev, s);
    if constexpr (kMaxGroups >= 8)
        if (g >= 8) return far_nw<T, 8, CPL>(lv, nlev, s);
    if constexpr (kMaxGroups >= 4)
        if (g >= 4) return far_nw<T, 4, CPL>(lv, nlev, s);
    if constexpr (kMaxGroups >= 2)
        if (g >= 2) return far_nw<T, 2, CPL>(lv, nlev, s);
    return far_nw<T, 1, CPL>(lv, nlev, s);
}

// Variant when the plan leaves it open, from measurements on MI355X:
//  * FP32 with 16-bit list entries: all 8 children per lane, in 4 parent groups per
//    workgroup, or 8 for levels of at least 256 parents (the 256^3 M2L 329 -> 269 us; the
//    128^3 one, 64 parents, stays fastest with 4: 53 us);
//  * FP64 with at least 64 parents: all children per lane in 4 groups (the 256^3 M2L
//    610 -> 527 us; with the halved kernel tile also the 128^3 one, 64 parents: 103 -> 99
//    us against 4 children per lane);
//  * levels of at least 256 parents with 32-bit entries (65535 or more intervals) as
//    with 16-bit ones (a 77^3-block cube of n = 6, p = 7: FP64 66 -> 62 ms per solve,
//    FP32 42 -> 36 ms);
//  * otherwise levels with at least 64 parents run 4 children per lane in 4 parent
//    groups; smaller levels 2 children per lane (more waves for little work) in 1 (FP64)
//    or 2 (FP32) groups.
// A launch over several levels takes the variant of its largest level.  Every variant
// computes the same bits.
template <typename T>
void m2l_default(int64_t nparents, bool idx16, int& waves, int& cpl) {
    if (sizeof(T) == 4 && (idx16 || nparents >= 256)) {
        if (waves == 0) waves = nparents >= 256 ? 8 : 4;
        if (cpl == 0) cpl = 8;
        return;
    }
    if (sizeof(T) == 8 && nparents >= 64) {
        if (waves == 0) waves = 4;
        if (cpl == 0) cpl = 8;
        return;
    }
    const bool big = nparents >= 64;
    if (waves == 0) waves = big ? 4 : (sizeof(T) == 8 ? 1 : 2);
    if (cpl == 0) cpl = big ? 4 : 2;
}

template <typename T>
hipError_t launch_prod_far_sib_levels(const FarLevel<T>* lv, int nlev, int waves, int cpl, hipStream_t s) {
    int64_t most = 0;
    int k = 0;
    bool idx16 = !m2l_wide_lists();
    for (int i = 0; i < nlev; ++i) {
        if (lv[i].nparents <= 0) continue;
        if (k != i || !chunk_fits_u32<T>(lv[i].nsrc + 1) || !sym_fits(lv[i].sym, lv[i].S))
            return hipErrorInvalidValue;  // empty levels only at the end
        most = lv[i].nparents > most ? lv[i].nparents : most;
        idx16 = idx16 && lv[i].nsrc < 65535;
        ++k;
    }
    if (k == 0) return hipSuccess;
    if (k > kMaxFarSegs) return hipErrorInvalidValue;
    const bool open = waves == 0 && cpl == 0;
    m2l_default<T>(most, idx16, waves, cpl);
    if (open && k > 1) {
        // with the variant left open, a level whose workgroups in the largest level's variant
        // would exceed half that level's count (many frequency chunks, few parents: the
        // 34-point levels of the lattice scheme) gets a launch of its own with its own
        // default variant; the others stay in one launch
        constexpr int F = M2LShape<T>::F;
        const int groups = std::min(waves, (sizeof(T) == 8 ? 8 : 16) / (8 / cpl));
        const int64_t ppg = (int64_t)M2LShape<T>::PPW * groups;
        auto wgs = [&](const FarLevel<T>& l) {
            return (int64_t)xcd_grid((l.S + F - 1) / F, 1) * ((l.nparents + ppg - 1) / ppg);
        };
        int64_t wmax = 0;
        for (int i = 0; i < k; ++i) wmax = std::max(wmax, wgs(lv[i]));
        FarLevel<T> keep[kMaxFarSegs];
        int nk = 0;
        for (int i = 0; i < k; ++i) {
            if (wgs(lv[i]) == wmax || 2 * wgs(lv[i]) <= wmax) {
                keep[nk++] = lv[i];
            } else {
                const hipError_t e = launch_prod_far_sib_levels<T>(&lv[i], 1, 0, 0, s);
                if (e != hipSuccess) return e;
            }
        }
        if (nk < k) return launch_prod_far_sib_levels<T>(keep, nk, waves, cpl, s);
    }
    switch (cpl) {
        case 8: return far_cpl<T, 8>(lv, k, waves, s);
        case 4: return far_cpl<T, 4>(lv, k, waves, s);
        case 2: return far_cpl<T, 2>(lv, k, waves, s);
        default: return far_cpl<T, 1>(lv, k, waves, s);
    }
}

template <typename T>
hipError_t launch_prod_far_sib(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* child8,
                               const int32_t* src216, cplx<T>* uhat, int64_t nparents, int64_t nitems, int64_t nsrc,
                               int S, int waves, int cpl, hipStream_t s, const SpecSym& sym) {
    if (nparents <= 0) return hipSuccess;
    const FarLevel<T> one{fhat, khat, child8, src216, uhat, nparents, nitems, nsrc, S, sym};
    return launch_prod_far_sib_levels<T>(&one, 1, waves, cpl, s);
}

template <typename T>
hipError_t launch_prod_far(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* ptr, const int32_t* src,
                           const int32_t* off, const int32_t* tgt, cplx<T>* uhat, int64_t ntgt, int64_t nitems,
                           int noff, int S, hipStream_t s, int64_t nsrc, const SpecSym& sym) {
    if (ntgt <= 0) return hipSuccess;
    if (nsrc < 0) nsrc = nitems;
    if (!sym_fits(sym, S)) return hipErrorInvalidValue;
    dim3 grid((unsigned)ntgt, (unsigned)((S + kProdThreads - 1) / kProdThreads));
    return lgf_launch(k_prod_far<T>, grid, dim3(kProdThreads), 0, s, fhat, khat, ptr, src, off, tgt, uhat, S,
                      (int)nitems, noff, (int)nsrc, sym);
}

#define LGF_INST(T)                                                                                              \
    template hipError_t launch_prod_near<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*,      \
                                            cplx<T>*, int64_t, int64_t, int64_t, int, int, int, hipStream_t,     \
                                            const SpecSym&);                                                     \
    template hipError_t launch_prod_far_sib<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*,   \
                                               cplx<T>*, int64_t, int64_t, int64_t, int, int, int, hipStream_t,  \
                                               const SpecSym&);                                                  \
    template hipError_t launch_prod_far_sib_levels<T>(const FarLevel<T>*, int, int, int, hipStream_t);           \
    template hipError_t launch_prod_far<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*,       \
                                           const int32_t*, const int32_t*, cplx<T>*, int64_t, int64_t, int, int, \
                                           hipStream_t, int64_t, const SpecSym&);
LGF_INST(double)
LGF_INST(float)
#undef LGF_INST

}  // namespace lgfdev
