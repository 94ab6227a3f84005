// Host side of the solver: layout validation, the octree of intervals and its lists
// (Sec. 3.1: RegSupp, IntrpSupp, InflList), 1D Lagrange matrices (Sec. 2.5), device
// workspace, the launch sequence of one solve (Steps 1-3) and the C ABI of lgf.h.
//
// Tree conventions: block coordinates are shifted so the bounding-box minimum is 0;
// the level-1 interval of block B has index B and the parent of interval I is
// floor(I / 2).  Interval I at level l spans [I s_l, (I+1) s_l]^3, s_l = n 2^(l-1), with
// nodes I s_l + k h_l, h_l = s_l / (p - 1), k in [0, p)^3.
// Lists: level 0 near neighbours |Q-P|_inf <= 1; level l < L: children of the parent's
// neighbours with |Q-P|_inf >= 2; top level L: every interval with |Q-P|_inf >= 2.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lgf.h"
#include "lgf_internal.h"

using namespace lgfdev;

namespace {

thread_local std::string t_err;

lgf_status fail(lgf_status st, const std::string& msg) {
    t_err = msg;
    return st;
}

inline uint64_t pack(int64_t x, int64_t y, int64_t z) {
    return (uint64_t)x | ((uint64_t)y << 21) | ((uint64_t)z << 42);
}

// Lagrange basis on nodes 0..p-1 evaluated at t
long double lagrange(int p, int k, long double t) {
    long double v = 1.0L;
    for (int j = 0; j < p; ++j)
        if (j != k) v *= (t - j) / (long double)(k - j);
    return v;
}

// zero fill by a kernel (no memset node, so the sequence stays graph-capturable)
__global__ void k_zero(int32_t* p, int64_t words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) p[i] = 0;
}

hipError_t zero_fill(void* p, int64_t bytes, hipStream_t s) {
    const int64_t words = bytes / 4;  // every buffer here is a multiple of 4 bytes
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, (int32_t*)p, words);
    return hipGetLastError();
}

struct DevBuf {
    void* ptr = nullptr;
    int64_t bytes = 0;
};

}  // namespace

struct LevelPlan {
    int64_t nint = 0;
    std::vector<int32_t> coords;    // [nint][3]
    std::vector<int32_t> parent;    // [nint] -> level l+1 (empty at the top)
    std::vector<int32_t> cpos;      // [nint] child position bits x | y<<1 | z<<2
    std::vector<int32_t> child8;    // [nint][8] children at level l-1 (levels >= 2)
    std::vector<int32_t> nbr27;     // [nint][27] same-level neighbours (levels >= 2)
    std::vector<int32_t> src216;    // [nint][216] children of the 27 neighbours (sentinel if absent)
    std::vector<int32_t> il_ptr, il_src, il_off;
    int radius = 3;
    std::shared_ptr<SpectraEntry> spectra;
    // device
    int32_t *d_parent = nullptr, *d_cpos = nullptr, *d_child8 = nullptr, *d_src216 = nullptr;
    bool sibling = false;  // level list served by the sibling-blocked kernel
    int32_t *d_ptr = nullptr, *d_src = nullptr, *d_off = nullptr;
    void *d_ftil = nullptr, *d_fhat = nullptr, *d_uhat = nullptr, *d_util = nullptr;
};

struct lgf_plan_s {
    int n = 0, p = 0, L = 0, Ltop = 0;
    lgf_precision prec = LGF_F64;
    int64_t nb = 0;
    std::vector<int32_t> blocks;
    std::vector<int32_t> nbr0;  // [nb][27]
    int64_t near_pairs = 0;
    std::vector<int32_t> g0_tgt8, g0_src64;  // level-0 target groups (2x2x2) and their 4^3 sources
    int64_t ngroups0 = 0;
    int32_t *d_g0_tgt8 = nullptr, *d_g0_src64 = nullptr;
    std::vector<LevelPlan> lv;  // index 0 unused, 1..L
    std::shared_ptr<SpectraEntry> spectra0;
    int32_t* d_nbr0 = nullptr;
    double *d_A = nullptr, *d_C01 = nullptr;
    void *d_fhat0 = nullptr, *d_uhat0 = nullptr;
    std::vector<DevBuf> allocs;
    int64_t ws_bytes = 0;
    int device = 0;
    // step profiling (events recorded on the solve stream)
    struct StepInfo {
        std::string name;
        double bytes, flops;
    };
    std::vector<StepInfo> steps;  // filled by the first profiled solve
    std::vector<hipEvent_t> events;
    int prof_max = 0, prof_solves = 0, prof_cursor = 0;
    bool prof_on = false;

    ~lgf_plan_s() {
        for (auto& b : allocs) hipFree(b.ptr);
        for (auto& e : events) hipEventDestroy(e);
        budget_release(ws_bytes);
    }
};

namespace {

template <typename P>
bool dev_alloc(lgf_plan_s* pl, P** out, int64_t bytes) {
    *out = nullptr;
    if (bytes <= 0) return true;
    void* ptr = nullptr;
    if (hipMalloc(&ptr, (size_t)bytes) != hipSuccess) return false;
    pl->allocs.push_back(DevBuf{ptr, bytes});
    *out = reinterpret_cast<P*>(ptr);
    return true;
}

// LGF_SYNC_CHECK=1 in the environment: synchronise after every launch and report the
// first failing step by name (debugging aid; off by default).
bool sync_check_enabled() {
    static const bool on = [] {
        const char* v = std::getenv("LGF_SYNC_CHECK");
        return v && v[0] == '1';
    }();
    return on;
}

hipError_t checked(hipError_t e, const char* what, hipStream_t s) {
    if (e == hipSuccess && sync_check_enabled()) {
        e = hipStreamSynchronize(s);
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e != hipSuccess) t_err = std::string(what) + ": " + hipGetErrorString(e);
    return e;
}

// Profiling: record an event after a step (and describe the step on the first solve).
struct Marker {
    lgf_plan_s* pl;
    hipStream_t s;
    bool on;
    int step = 0;
    Marker(lgf_plan_s* p, hipStream_t st) : pl(p), s(st) {
        on = pl->prof_on && pl->prof_solves < pl->prof_max;
        if (on) {
            if (pl->prof_solves == 0) pl->steps.clear();
            hipEventRecord(pl->events[pl->prof_cursor++], s);
        }
    }
    void operator()(const std::string& name, double bytes, double flops) {
        if (!on) return;
        if (pl->prof_solves == 0) pl->steps.push_back({name, bytes, flops});
        hipEventRecord(pl->events[pl->prof_cursor++], s);
        ++step;
    }
    void finish() {
        if (on) ++pl->prof_solves;
    }
};

inline double fft_flops(int M) {  // Table 1: 2 (8 N_b) log2(8 N_b) for a padded M^3 transform
    const double N = (double)M * M * M;
    return 2.0 * N * std::log2(N);
}

template <typename T>
hipError_t run_solve(lgf_plan_s* pl, const T* f, T* u, hipStream_t s) {
    using C = cplx<T>;
    using U = typename FarAcc<T>::type;
    const int n = pl->n, p = pl->p;
    hipError_t e;
    Marker mark(pl, s);
    const double es = sizeof(T), cs = 2.0 * sizeof(T);
    const double n3 = (double)n * n * n, p3 = (double)p * p * p;
    const double S0 = pl->spectra0->S, S1 = (double)(2 * p) * (2 * p) * (p + 1);
    const double nb = (double)pl->nb;
    auto lvN = [&](int l) { return (double)pl->lv[l].nint; };
#define LGF_CHECK(x)                                      \
    do {                                                  \
        if ((e = checked((x), #x, s)) != hipSuccess) return e; \
    } while (0)
    LGF_CHECK(launch_pad_fft<T>(n, f, (C*)pl->d_fhat0, pl->nb, s));
    mark("fft_fwd_l0", nb * (n3 * es + S0 * cs), nb * fft_flops(2 * n));
    if (pl->Ltop >= 1) {
        LGF_CHECK(launch_reg_block<T>(f, pl->d_A, (T*)pl->lv[1].d_ftil, pl->nb, n, p, s));
        mark("reg_l0_l1", nb * (n3 + p3) * es, nb * 2.0 * (p * n3 + p * p * n * n + p3 * n));
        for (int l = 1; l < pl->Ltop; ++l) {
            LGF_CHECK(launch_reg_up<T>((const T*)pl->lv[l].d_ftil, pl->lv[l + 1].d_child8, pl->d_C01,
                                       (T*)pl->lv[l + 1].d_ftil, pl->lv[l + 1].nint, p, s));
            mark("reg_l" + std::to_string(l) + "_l" + std::to_string(l + 1), (lvN(l) + lvN(l + 1)) * p3 * es,
                 lvN(l) * 2.0 * 3.0 * p3 * p);
        }
        for (int l = 1; l <= pl->Ltop; ++l)
            if (!pl->lv[l].il_src.empty()) {
                LGF_CHECK(launch_pad_fft<T>(p, (const T*)pl->lv[l].d_ftil, (C*)pl->lv[l].d_fhat, pl->lv[l].nint, s));
                mark("fft_fwd_l" + std::to_string(l), lvN(l) * (p3 * es + S1 * cs), lvN(l) * fft_flops(2 * p));
            }
    }
    LGF_CHECK(launch_prod_near<T>((const C*)pl->d_fhat0, (const C*)pl->spectra0->dev, pl->d_g0_tgt8, pl->d_g0_src64,
                                  (C*)pl->d_uhat0, pl->ngroups0, pl->nb, pl->spectra0->S, s));
    mark("prod_l0", (2.0 * nb + 27.0) * S0 * cs, (double)pl->near_pairs * S0 * 8.0);
    for (int l = 1; l <= pl->Ltop; ++l) {
        LevelPlan& L = pl->lv[l];
        if (L.il_src.empty()) continue;
        if (L.sibling) {
            const LevelPlan& Pp = pl->lv[l + 1];
            LGF_CHECK(launch_prod_far_sib<T>((const C*)L.d_fhat, (const C*)L.spectra->dev, Pp.d_child8, Pp.d_src216,
                                             (C*)L.d_uhat, Pp.nint, L.nint, L.spectra->S, s));
        } else {
            LGF_CHECK(launch_prod_far<T>((const C*)L.d_fhat, (const C*)L.spectra->dev, L.d_ptr, L.d_src, L.d_off,
                                         (C*)L.d_uhat, L.nint, L.spectra->noff, L.spectra->S, s));
        }
        mark("prod_l" + std::to_string(l), (2.0 * lvN(l) + 316.0) * S1 * cs, (double)L.il_src.size() * S1 * 8.0);
    }
    for (int l = pl->Ltop; l >= 1; --l) {
        LevelPlan& L = pl->lv[l];
        if (L.il_src.empty()) {
            LGF_CHECK(zero_fill(L.d_util, L.nint * (int64_t)p * p * p * sizeof(U), s));
            mark("zero_l" + std::to_string(l), lvN(l) * p3 * es, 0.0);
        } else {
            LGF_CHECK((launch_ifft_trunc<T, U, U>(p, (const C*)L.d_uhat, (U*)L.d_util, L.nint, s)));
            mark("fft_inv_l" + std::to_string(l), lvN(l) * (S1 * cs + p3 * es), lvN(l) * fft_flops(2 * p));
        }
        if (l < pl->Ltop) {
            LGF_CHECK(launch_interp_down<U>((const U*)pl->lv[l + 1].d_util, pl->lv[l + 1].d_child8, pl->d_C01,
                                            (U*)L.d_util, pl->lv[l + 1].nint, p, s));
            mark("interp_l" + std::to_string(l + 1) + "_l" + std::to_string(l), (lvN(l + 1) + 2.0 * lvN(l)) * p3 * es,
                 lvN(l) * 2.0 * 3.0 * p3 * p);
        }
    }
    LGF_CHECK((launch_ifft_trunc<T, T, T>(n, (const C*)pl->d_uhat0, u, pl->nb, s)));
    mark("fft_inv_l0", nb * (S0 * cs + n3 * es), nb * fft_flops(2 * n));
    if (pl->Ltop >= 1) {
        LGF_CHECK((launch_final<T, U>(u, (const U*)pl->lv[1].d_util, pl->d_A, u, pl->nb, n, p, s)));
        mark("final_l1_l0", nb * (2.0 * n3 + p3) * es, nb * 2.0 * (p3 * n + p * p * n * n + p * n3));
    }
    mark.finish();
#undef LGF_CHECK
    return hipSuccess;
}

lgf_status build_plan(const int32_t* ijk, int64_t nblocks, int n, int p, int levels, lgf_precision prec,
                      hipStream_t s, lgf_plan_s* pl) {
    pl->n = n;
    pl->p = p;
    pl->prec = prec;
    pl->nb = nblocks;
    hipGetDevice(&pl->device);
    // ---- layout: shift to the bounding-box minimum, reject duplicates and huge spans
    int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    for (int64_t b = 0; b < nblocks; ++b)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min<int64_t>(lo[d], ijk[3 * b + d]);
            hi[d] = std::max<int64_t>(hi[d], ijk[3 * b + d]);
        }
    int64_t ext = 1;
    for (int d = 0; d < 3; ++d) {
        if (hi[d] - lo[d] >= (1 << 20)) return fail(LGF_ERR_LAYOUT, "layout spans more than 2^20 blocks");
        ext = std::max<int64_t>(ext, hi[d] - lo[d] + 1);
    }
    pl->blocks.resize(3 * nblocks);
    std::unordered_map<uint64_t, int32_t> idx0;
    idx0.reserve(nblocks * 2);
    for (int64_t b = 0; b < nblocks; ++b) {
        for (int d = 0; d < 3; ++d) pl->blocks[3 * b + d] = (int32_t)(ijk[3 * b + d] - lo[d]);
        const uint64_t key = pack(pl->blocks[3 * b], pl->blocks[3 * b + 1], pl->blocks[3 * b + 2]);
        if (!idx0.emplace(key, (int32_t)b).second) return fail(LGF_ERR_LAYOUT, "duplicate block in layout");
    }
    int full = 1;
    while ((int64_t(1) << (full - 1)) < ext) ++full;
    pl->L = levels <= 0 ? full : std::min(levels, full);
    if (pl->L >= kMaxLevels) return fail(LGF_ERR_LAYOUT, "tree deeper than supported");

    // ---- level 0 near-neighbour table
    pl->nbr0.assign(27 * nblocks, -1);
    for (int64_t b = 0; b < nblocks; ++b) {
        const int32_t* P = &pl->blocks[3 * b];
        for (int d = 0; d < 27; ++d) {
            const int Dx = d % 3 - 1, Dy = (d / 3) % 3 - 1, Dz = d / 9 - 1;
            const int64_t qx = P[0] - Dx, qy = P[1] - Dy, qz = P[2] - Dz;  // Q = P - D
            if (qx < 0 || qy < 0 || qz < 0) continue;
            auto it = idx0.find(pack(qx, qy, qz));
            if (it != idx0.end()) {
                pl->nbr0[27 * b + d] = it->second;
                ++pl->near_pairs;
            }
        }
    }
    // ---- level-0 target groups: blocks 2J + c, sources 2J + (-1..2)^3
    {
        std::unordered_map<uint64_t, int32_t> gidx;
        for (int64_t b = 0; b < nblocks; ++b) {
            const int32_t* P = &pl->blocks[3 * b];
            const uint64_t key = pack(P[0] >> 1, P[1] >> 1, P[2] >> 1);
            auto it = gidx.find(key);
            int32_t g;
            if (it == gidx.end()) {
                g = (int32_t)pl->ngroups0++;
                gidx.emplace(key, g);
                pl->g0_tgt8.resize(8 * pl->ngroups0, -1);
                pl->g0_src64.resize(64 * pl->ngroups0, (int32_t)nblocks);  // zero sentinel item
                for (int sidx = 0; sidx < 64; ++sidx) {
                    const int64_t qx = 2 * (int64_t)(P[0] >> 1) + (sidx & 3) - 1;
                    const int64_t qy = 2 * (int64_t)(P[1] >> 1) + ((sidx >> 2) & 3) - 1;
                    const int64_t qz = 2 * (int64_t)(P[2] >> 1) + (sidx >> 4) - 1;
                    if (qx < 0 || qy < 0 || qz < 0) continue;
                    auto jt = idx0.find(pack(qx, qy, qz));
                    if (jt != idx0.end()) pl->g0_src64[64 * g + sidx] = jt->second;
                }
            } else {
                g = it->second;
            }
            pl->g0_tgt8[8 * g + ((P[0] & 1) | ((P[1] & 1) << 1) | ((P[2] & 1) << 2))] = (int32_t)b;
        }
    }
    // ---- levels: coordinates, parents, children
    pl->lv.assign(pl->L + 1, LevelPlan());
    std::vector<std::unordered_map<uint64_t, int32_t>> idx(pl->L + 2);
    pl->lv[1].nint = nblocks;
    pl->lv[1].coords = pl->blocks;
    idx[1] = idx0;
    for (int l = 1; l < pl->L; ++l) {
        LevelPlan& C = pl->lv[l];
        LevelPlan& P = pl->lv[l + 1];
        C.parent.resize(C.nint);
        C.cpos.resize(C.nint);
        for (int64_t i = 0; i < C.nint; ++i) {
            const int32_t x = C.coords[3 * i], y = C.coords[3 * i + 1], z = C.coords[3 * i + 2];
            const uint64_t key = pack(x >> 1, y >> 1, z >> 1);
            auto it = idx[l + 1].find(key);
            int32_t j;
            if (it == idx[l + 1].end()) {
                j = (int32_t)P.nint++;
                idx[l + 1].emplace(key, j);
                P.coords.push_back(x >> 1);
                P.coords.push_back(y >> 1);
                P.coords.push_back(z >> 1);
            } else {
                j = it->second;
            }
            C.parent[i] = j;
            C.cpos[i] = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
        }
        P.child8.assign(8 * P.nint, -1);
        for (int64_t i = 0; i < C.nint; ++i) P.child8[8 * C.parent[i] + C.cpos[i]] = (int32_t)i;
    }
    for (int l = 2; l <= pl->L; ++l) {
        LevelPlan& Lv = pl->lv[l];
        Lv.nbr27.assign(27 * Lv.nint, -1);
        for (int64_t i = 0; i < Lv.nint; ++i)
            for (int e = 0; e < 27; ++e) {
                const int64_t jx = Lv.coords[3 * i] + e % 3 - 1, jy = Lv.coords[3 * i + 1] + (e / 3) % 3 - 1,
                              jz = Lv.coords[3 * i + 2] + e / 9 - 1;
                if (jx < 0 || jy < 0 || jz < 0) continue;
                auto it = idx[l].find(pack(jx, jy, jz));
                if (it != idx[l].end()) Lv.nbr27[27 * i + e] = it->second;
            }
        const int32_t sentinel = (int32_t)pl->lv[l - 1].nint;
        Lv.src216.assign(216 * Lv.nint, sentinel);
        for (int64_t i = 0; i < Lv.nint; ++i)
            for (int e = 0; e < 27; ++e) {
                const int32_t Jn = Lv.nbr27[27 * i + e];
                if (Jn < 0) continue;
                for (int cs = 0; cs < 8; ++cs) {
                    const int32_t q = Lv.child8[8 * Jn + cs];
                    if (q >= 0) Lv.src216[216 * i + 8 * e + cs] = q;
                }
            }
    }
    // ---- interaction lists
    for (int l = 1; l <= pl->L; ++l) {
        LevelPlan& Lv = pl->lv[l];
        Lv.il_ptr.assign(Lv.nint + 1, 0);
        int maxd = 0;
        std::vector<std::pair<int32_t, int32_t>> tmp;  // (src, D packed later)
        std::vector<int32_t> src, offs;
        std::vector<std::array<int32_t, 3>> dvec;
        for (int64_t i = 0; i < Lv.nint; ++i) {
            const int32_t* P = &Lv.coords[3 * i];
            std::vector<std::pair<int64_t, std::array<int32_t, 3>>> cand;  // (q, D)
            if (l < pl->L) {
                const int32_t* Pp = &pl->lv[l + 1].coords[3 * Lv.parent[i]];
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int64_t jx = Pp[0] + dx, jy = Pp[1] + dy, jz = Pp[2] + dz;
                            if (jx < 0 || jy < 0 || jz < 0) continue;
                            auto it = idx[l + 1].find(pack(jx, jy, jz));
                            if (it == idx[l + 1].end()) continue;
                            for (int c = 0; c < 8; ++c) {
                                const int32_t q = pl->lv[l + 1].child8[8 * it->second + c];
                                if (q < 0) continue;
                                const int32_t* Q = &Lv.coords[3 * q];
                                std::array<int32_t, 3> D{P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
                                const int dinf = std::max(std::abs(D[0]), std::max(std::abs(D[1]), std::abs(D[2])));
                                if (dinf >= 2) cand.push_back({q, D});
                            }
                        }
            } else {
                for (int64_t q = 0; q < Lv.nint; ++q) {
                    const int32_t* Q = &Lv.coords[3 * q];
                    std::array<int32_t, 3> D{P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
                    const int dinf = std::max(std::abs(D[0]), std::max(std::abs(D[1]), std::abs(D[2])));
                    if (dinf >= 2) cand.push_back({q, D});
                }
            }
            std::sort(cand.begin(), cand.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
            for (const auto& cd : cand) {
                src.push_back((int32_t)cd.first);
                dvec.push_back(cd.second);
                maxd = std::max(maxd, std::max(std::abs(cd.second[0]), std::max(std::abs(cd.second[1]), std::abs(cd.second[2]))));
            }
            Lv.il_ptr[i + 1] = (int32_t)src.size();
        }
        Lv.radius = std::max(3, maxd);
        const int R = Lv.radius, W = 2 * R + 1;
        Lv.il_src = src;
        Lv.il_off.resize(src.size());
        for (size_t e = 0; e < src.size(); ++e)
            Lv.il_off[e] = (dvec[e][0] + R) + W * ((dvec[e][1] + R) + W * (dvec[e][2] + R));
        if (!src.empty()) pl->Ltop = l;
        Lv.sibling = (l < pl->L) && !src.empty();
    }
    if (pl->Ltop >= 1 && (int64_t)(2 * pl->lv[pl->Ltop].radius + 1) * (2 * pl->lv[pl->Ltop].radius + 1) *
                                 (2 * pl->lv[pl->Ltop].radius + 1) > 300000)
        return fail(LGF_ERR_LAYOUT, "top-level interaction offsets too large: use more levels");

    // ---- kernel spectra (shared cache)
    std::string err;
    const int ip = prec == LGF_F64 ? 0 : 1;
    pl->spectra0 = get_spectra(SpectraKey{n, p, 0, 1, ip}, s, err);
    if (!pl->spectra0) return fail(err.find("budget") != std::string::npos ? LGF_ERR_BUDGET : LGF_ERR_DEVICE, err);
    for (int l = 1; l <= pl->Ltop; ++l) {
        if (pl->lv[l].il_src.empty()) continue;
        pl->lv[l].spectra = get_spectra(SpectraKey{n, p, l, pl->lv[l].radius, ip}, s, err);
        if (!pl->lv[l].spectra)
            return fail(err.find("budget") != std::string::npos ? LGF_ERR_BUDGET : LGF_ERR_DEVICE, err);
    }

    // ---- matrices (FP64)
    std::vector<double> A(p * n), C01(2 * p * p);
    for (int k = 0; k < p; ++k)
        for (int j = 0; j < n; ++j) A[k * n + j] = (double)lagrange(p, k, (long double)j * (p - 1) / n);
    for (int c = 0; c < 2; ++c)
        for (int mm = 0; mm < p; ++mm)
            for (int k = 0; k < p; ++k)
                C01[c * p * p + mm * p + k] = (double)lagrange(p, mm, (long double)(c * (p - 1) + k) / 2.0L);

    // ---- device memory
    const size_t esz = prec == LGF_F64 ? sizeof(double) : sizeof(float);
    const int64_t S0 = spec_padded(pl->spectra0->S);
    const int M1 = 2 * p;
    const int64_t S1 = spec_padded(M1 * M1 * (M1 / 2 + 1));
    const int64_t p3 = (int64_t)p * p * p;
    const int64_t usz = 8;  // far-field down-pass values: double or float-float
    const int topc = std::min(pl->Ltop + 1, pl->L);  // highest level whose child8 / nbr27 is used
    int64_t need = 27 * nblocks * 4 + pl->ngroups0 * 72 * 4 + (p * n + 2 * p * p) * 8 + (2 * nblocks + 1) * S0 * 2 * esz;
    for (int l = 1; l <= pl->Ltop; ++l) {
        const LevelPlan& Lv = pl->lv[l];
        need += Lv.nint * (p3 * (esz + usz) + 2 * 4) + (Lv.nint + 1) * 4 + Lv.il_src.size() * 8;
        if (!Lv.il_src.empty()) need += (2 * Lv.nint + 1) * S1 * 2 * esz;
    }
    for (int l = 2; l <= topc && pl->Ltop >= 1; ++l) need += pl->lv[l].nint * 224 * 4;
    if (!budget_reserve(need)) return fail(LGF_ERR_BUDGET, "plan workspace exceeds the device-memory budget");
    pl->ws_bytes = need;
    bool ok = dev_alloc(pl, &pl->d_nbr0, 27 * nblocks * 4) && dev_alloc(pl, &pl->d_g0_tgt8, pl->ngroups0 * 8 * 4) &&
              dev_alloc(pl, &pl->d_g0_src64, pl->ngroups0 * 64 * 4) && dev_alloc(pl, &pl->d_A, p * n * 8) &&
              dev_alloc(pl, &pl->d_C01, 2 * p * p * 8) && dev_alloc(pl, &pl->d_fhat0, (nblocks + 1) * S0 * 2 * esz) &&
              dev_alloc(pl, &pl->d_uhat0, nblocks * S0 * 2 * esz);
    for (int l = 1; ok && l <= pl->Ltop; ++l) {
        LevelPlan& Lv = pl->lv[l];
        ok = dev_alloc(pl, &Lv.d_ftil, Lv.nint * p3 * esz) && dev_alloc(pl, &Lv.d_util, Lv.nint * p3 * usz);
        if (ok && l < pl->Ltop)
            ok = dev_alloc(pl, &Lv.d_parent, Lv.nint * 4) && dev_alloc(pl, &Lv.d_cpos, Lv.nint * 4);
        if (ok && !Lv.il_src.empty())
            ok = dev_alloc(pl, &Lv.d_ptr, (Lv.nint + 1) * 4) && dev_alloc(pl, &Lv.d_src, Lv.il_src.size() * 4) &&
                 dev_alloc(pl, &Lv.d_off, Lv.il_src.size() * 4) &&
                 dev_alloc(pl, &Lv.d_fhat, (Lv.nint + 1) * S1 * 2 * esz) &&
                 dev_alloc(pl, &Lv.d_uhat, Lv.nint * S1 * 2 * esz);
    }
    for (int l = 2; ok && l <= topc && pl->Ltop >= 1; ++l)
        ok = dev_alloc(pl, &pl->lv[l].d_child8, pl->lv[l].nint * 32) &&
             dev_alloc(pl, &pl->lv[l].d_src216, pl->lv[l].nint * 216 * 4);
    if (!ok) return fail(LGF_ERR_OOM, "device allocation failed for the plan workspace");
    hipError_t e = hipMemcpyAsync(pl->d_nbr0, pl->nbr0.data(), 27 * nblocks * 4, hipMemcpyHostToDevice, s);
    e = e == hipSuccess ? hipMemcpyAsync(pl->d_g0_tgt8, pl->g0_tgt8.data(), pl->g0_tgt8.size() * 4,
                                         hipMemcpyHostToDevice, s) : e;
    e = e == hipSuccess ? hipMemcpyAsync(pl->d_g0_src64, pl->g0_src64.data(), pl->g0_src64.size() * 4,
                                         hipMemcpyHostToDevice, s) : e;
    e = e == hipSuccess ? hipMemcpyAsync(pl->d_A, A.data(), A.size() * 8, hipMemcpyHostToDevice, s) : e;
    e = e == hipSuccess ? hipMemcpyAsync(pl->d_C01, C01.data(), C01.size() * 8, hipMemcpyHostToDevice, s) : e;
    for (int l = 1; e == hipSuccess && l <= pl->Ltop; ++l) {
        LevelPlan& Lv = pl->lv[l];
        if (Lv.d_parent) e = hipMemcpyAsync(Lv.d_parent, Lv.parent.data(), Lv.nint * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && Lv.d_cpos)
            e = hipMemcpyAsync(Lv.d_cpos, Lv.cpos.data(), Lv.nint * 4, hipMemcpyHostToDevice, s);

        if (e == hipSuccess && Lv.d_ptr) {
            e = hipMemcpyAsync(Lv.d_ptr, Lv.il_ptr.data(), (Lv.nint + 1) * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(Lv.d_src, Lv.il_src.data(), Lv.il_src.size() * 4, hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(Lv.d_off, Lv.il_off.data(), Lv.il_off.size() * 4, hipMemcpyHostToDevice, s);
        }
    }
    for (int l = 2; e == hipSuccess && l <= topc && pl->Ltop >= 1; ++l) {
        LevelPlan& Lv = pl->lv[l];
        e = hipMemcpyAsync(Lv.d_child8, Lv.child8.data(), Lv.nint * 32, hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(Lv.d_src216, Lv.src216.data(), Lv.nint * 216 * 4, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = zero_fill(pl->d_fhat0, (nblocks + 1) * S0 * 2 * esz, s);
    for (int l = 1; e == hipSuccess && l <= pl->Ltop; ++l)
        if (pl->lv[l].d_fhat) e = zero_fill(pl->lv[l].d_fhat, (pl->lv[l].nint + 1) * S1 * 2 * esz, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(LGF_ERR_DEVICE, std::string("plan upload failed: ") + hipGetErrorString(e));
    return LGF_OK;
}

}  // namespace

// ============================================================== memory budget
namespace lgfdev {
static std::atomic<int64_t> g_budget{0}, g_used{0};
bool budget_reserve(int64_t bytes) {
    int64_t cur = g_used.load();
    for (;;) {
        const int64_t b = g_budget.load();
        if (b > 0 && cur + bytes > b) return false;
        if (g_used.compare_exchange_weak(cur, cur + bytes)) return true;
    }
}
void budget_release(int64_t bytes) { g_used.fetch_sub(bytes); }
int64_t budget_in_use() { return g_used.load(); }
void budget_set(int64_t bytes) { g_budget.store(bytes); }
}  // namespace lgfdev

// ============================================================== C ABI
extern "C" {

lgf_status lgf_plan_create(const int32_t* block_ijk, int64_t nblocks, int32_t n, int32_t p, int32_t levels,
                           lgf_precision prec, void* hip_stream, lgf_plan_t* out) {
    t_err.clear();
    if (!out) return fail(LGF_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!block_ijk) return fail(LGF_ERR_ARG, "block_ijk is NULL");
    if (nblocks < 1) return fail(LGF_ERR_LAYOUT, "empty layout");
    if (nblocks > (int64_t)1 << 30) return fail(LGF_ERR_ARG, "too many blocks");
    if (n != 4 && n != 8 && n != 16) return fail(LGF_ERR_ARG, "n must be 4, 8 or 16");
    if (p < 2 || p > 10) return fail(LGF_ERR_ARG, "p must lie in [2, 10]");
    if (prec != LGF_F64 && prec != LGF_F32) return fail(LGF_ERR_ARG, "unknown precision");
    lgf_plan_s* pl = nullptr;
    try {
        pl = new lgf_plan_s();
        lgf_status st = build_plan(block_ijk, nblocks, n, p, levels, prec, (hipStream_t)hip_stream, pl);
        if (st != LGF_OK) {
            delete pl;
            return st;
        }
    } catch (const std::bad_alloc&) {
        delete pl;
        return fail(LGF_ERR_OOM, "host allocation failed");
    } catch (...) {
        delete pl;
        return fail(LGF_ERR_DEVICE, "unexpected failure while building the plan");
    }
    *out = pl;
    return LGF_OK;
}

lgf_status lgf_solve(lgf_plan_t plan, const void* f, void* u, void* hip_stream) {
    if (!plan || !f || !u) return fail(LGF_ERR_ARG, "NULL argument to lgf_solve");
    t_err.clear();
    hipError_t e = plan->prec == LGF_F64
                       ? run_solve<double>(plan, (const double*)f, (double*)u, (hipStream_t)hip_stream)
                       : run_solve<float>(plan, (const float*)f, (float*)u, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(LGF_ERR_DEVICE, std::string("solve failed at ") + t_err);
    return LGF_OK;
}

lgf_status lgf_solve_many(const lgf_plan_t* plans, const void* const* f, void* const* u, int32_t count,
                          void* hip_stream) {
    if (count < 0 || (count > 0 && (!plans || !f || !u))) return fail(LGF_ERR_ARG, "bad arguments to lgf_solve_many");
    for (int32_t i = 0; i < count; ++i)
        for (int32_t j = 0; j < i; ++j)
            if (plans[i] == plans[j]) return fail(LGF_ERR_ARG, "lgf_solve_many: a plan appears twice");
    for (int32_t i = 0; i < count; ++i) {
        lgf_status st = lgf_solve(plans[i], f[i], u[i], hip_stream);
        if (st != LGF_OK) return st;
    }
    return LGF_OK;
}

lgf_status lgf_plan_query(lgf_plan_t plan, lgf_plan_info* info) {
    if (!plan || !info) return fail(LGF_ERR_ARG, "NULL argument to lgf_plan_query");
    std::memset(info, 0, sizeof(*info));
    info->nblocks = plan->nb;
    info->npoints = plan->nb * (int64_t)plan->n * plan->n * plan->n;
    info->n = plan->n;
    info->p = plan->p;
    info->levels = plan->L;
    info->top_level = plan->Ltop;
    info->near_pairs = plan->near_pairs;
    for (int l = 1; l <= plan->L && l < 16; ++l) {
        info->far_pairs[l] = (int64_t)plan->lv[l].il_src.size();
        info->intervals[l] = plan->lv[l].nint;
    }
    info->intervals[0] = plan->nb;
    info->workspace_bytes = plan->ws_bytes;
    int64_t sb = plan->spectra0 ? plan->spectra0->bytes : 0;
    for (int l = 1; l <= plan->Ltop; ++l)
        if (plan->lv[l].spectra) sb += plan->lv[l].spectra->bytes;
    info->spectra_bytes = sb;
    info->precision = plan->prec;
    return LGF_OK;
}

lgf_status lgf_plan_destroy(lgf_plan_t plan) {
    delete plan;
    return LGF_OK;
}

lgf_status lgf_set_memory_budget(int64_t bytes) {
    if (bytes < 0) return fail(LGF_ERR_ARG, "negative budget");
    budget_set(bytes);
    return LGF_OK;
}

int64_t lgf_memory_in_use(void) { return budget_in_use(); }

lgf_status lgf_spectra_cache_trim(void) {
    spectra_trim();
    return LGF_OK;
}

const char* lgf_last_error(void) { return t_err.c_str(); }

lgf_status lgf_profile_enable(lgf_plan_t plan, int32_t max_solves) {
    if (!plan || max_solves < 1) return fail(LGF_ERR_ARG, "lgf_profile_enable: bad arguments");
    const size_t need = (size_t)max_solves * (LGF_MAX_STEPS + 1);
    while (plan->events.size() < need) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return fail(LGF_ERR_DEVICE, "hipEventCreate failed");
        plan->events.push_back(ev);
    }
    plan->prof_max = max_solves;
    plan->prof_solves = 0;
    plan->prof_cursor = 0;
    plan->prof_on = true;
    return LGF_OK;
}

lgf_status lgf_profile_collect(lgf_plan_t plan, lgf_step_profile* out, double* solve_ms, int32_t max_out) {
    if (!plan || !out) return fail(LGF_ERR_ARG, "lgf_profile_collect: bad arguments");
    std::memset(out, 0, sizeof(*out));
    plan->prof_on = false;
    const int ns = (int)plan->steps.size();
    if (ns > LGF_MAX_STEPS) return fail(LGF_ERR_ARG, "too many steps");
    out->nsteps = ns;
    out->nsolves = plan->prof_solves;
    if (plan->prof_cursor > 0 && hipEventSynchronize(plan->events[plan->prof_cursor - 1]) != hipSuccess)
        return fail(LGF_ERR_DEVICE, "hipEventSynchronize failed");
    for (int j = 0; j < ns; ++j) {
        std::snprintf(out->name[j], sizeof(out->name[j]), "%s", plan->steps[j].name.c_str());
        out->bytes[j] = plan->steps[j].bytes;
        out->flops[j] = plan->steps[j].flops;
    }
    for (int i = 0; i < plan->prof_solves; ++i) {
        hipEvent_t* ev = &plan->events[(size_t)i * (ns + 1)];
        for (int j = 0; j < ns; ++j) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[j], ev[j + 1]) != hipSuccess)
                return fail(LGF_ERR_DEVICE, "hipEventElapsedTime failed");
            out->total_ms[j] += ms;
        }
        if (solve_ms && i < max_out) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, ev[0], ev[ns]);
            solve_ms[i] = ms;
        }
    }
    plan->prof_solves = 0;
    plan->prof_cursor = 0;
    return LGF_OK;
}

lgf_status lgf_green_table(int32_t R, double* out) {
    if (R < 1 || R > 128 || !out) return fail(LGF_ERR_ARG, "lgf_green_table: R must be in [1, 128]");
    std::string err;
    const int Rt = std::max<int>(R, 2);
    const double* G = green_table_device(Rt, nullptr, err);
    if (!G) return fail(LGF_ERR_DEVICE, err);
    std::vector<double> full((size_t)Rt * Rt * Rt);
    if (hipMemcpy(full.data(), G, full.size() * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(LGF_ERR_DEVICE, "copy of the Green's function table failed");
    for (int a = 0; a < R; ++a)
        for (int b = 0; b < R; ++b)
            for (int c = 0; c < R; ++c) out[((size_t)a * R + b) * R + c] = full[((size_t)a * Rt + b) * Rt + c];
    return LGF_OK;
}

lgf_status lgf_far_kernel(const double* pts, int64_t npts, double* out) {
    if (npts < 0 || (npts > 0 && (!pts || !out))) return fail(LGF_ERR_ARG, "lgf_far_kernel: bad arguments");
    if (npts == 0) return LGF_OK;
    double *dp = nullptr, *dout = nullptr;
    if (hipMalloc(&dp, npts * 3 * 8) != hipSuccess || hipMalloc(&dout, npts * 8) != hipSuccess) {
        if (dp) hipFree(dp);
        return fail(LGF_ERR_OOM, "lgf_far_kernel: device allocation failed");
    }
    std::string err;
    hipError_t e = hipMemcpy(dp, pts, npts * 3 * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = far_kernel_device(dp, npts, dout, nullptr, err);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out, dout, npts * 8, hipMemcpyDeviceToHost);
    hipFree(dp);
    hipFree(dout);
    if (e != hipSuccess) return fail(LGF_ERR_DEVICE, err.empty() ? hipGetErrorString(e) : err);
    return LGF_OK;
}

}  // extern "C"
