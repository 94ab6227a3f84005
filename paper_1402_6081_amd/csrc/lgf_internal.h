// Internal declarations shared by the library's translation units (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <algorithm>
#include <mutex>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/lgf.h"
#include "lgf_device.h"
#include "lgf_host.h"

namespace lgfdev {

// ------------------------------------------------------------------ launches and graph recording
// Every kernel launch of a solve goes through lgf_launch.  Normally it is an ordinary launch on
// the stream.  While a GraphRecorder is active on the calling thread (lgf_graph_create), the
// launch becomes an explicit kernel node of the recorder's graph instead: its argument block is
// allocated by the recorder and outlives the graph, its dependencies are the last nodes issued on
// the same stream, and event records and waits between streams (rec_event_record /
// rec_stream_wait) become dependency edges.  No stream capture is involved and no node is copied.
struct GraphRecorder {
    struct ArgBlock {
        virtual ~ArgBlock() = default;
    };
    template <typename Tuple>
    struct Args : ArgBlock {
        Tuple values;
        std::vector<void*> ptrs;
        explicit Args(Tuple&& t) : values(std::move(t)) {}
    };
    hipGraph_t graph = nullptr;
    std::map<hipStream_t, std::vector<hipGraphNode_t>> tails;  // nodes the next launch on a stream follows
    std::map<hipEvent_t, std::vector<hipGraphNode_t>> events;  // nodes an event was recorded behind
    std::vector<std::unique_ptr<ArgBlock>> args;               // argument blocks of the nodes
    int64_t launches = 0;                                       // kernel nodes added
    hipError_t err = hipSuccess;                                // first failure (sticky)
};
GraphRecorder* active_recorder();  // the calling thread's recorder, or nullptr

template <typename Tuple, size_t... I>
void arg_pointers(Tuple& t, std::vector<void*>& p, std::index_sequence<I...>) {
    p = {static_cast<void*>(&std::get<I>(t))...};
}

// Arguments are converted to the kernel's parameter types first; the launch passes one
// pointer per parameter (hipLaunchKernel), the graph node the same pointers.
template <typename... Params, typename... Args>
hipError_t lgf_launch(void (*kernel)(Params...), dim3 grid, dim3 block, size_t shmem, hipStream_t s,
                      Args&&... args) {
    static_assert(sizeof...(Params) == sizeof...(Args), "kernel argument count");
    static_assert(sizeof...(Params) > 0, "kernels here take arguments");
    using Tuple = std::tuple<std::decay_t<Params>...>;
    GraphRecorder* r = active_recorder();
    if (!r) {
        Tuple vals(static_cast<std::decay_t<Params>>(args)...);
        std::array<void*, sizeof...(Params)> ptrs = std::apply(
            [](auto&... v) { return std::array<void*, sizeof...(Params)>{static_cast<void*>(&v)...}; }, vals);
        return hipLaunchKernel(reinterpret_cast<const void*>(kernel), grid, block, ptrs.data(), shmem, s);
    }
    if (r->err != hipSuccess) return r->err;
    auto blk = std::make_unique<GraphRecorder::Args<Tuple>>(Tuple(static_cast<std::decay_t<Params>>(args)...));
    arg_pointers(blk->values, blk->ptrs, std::index_sequence_for<Params...>{});
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(kernel);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = (unsigned)shmem;
    kp.kernelParams = blk->ptrs.empty() ? nullptr : blk->ptrs.data();
    kp.extra = nullptr;
    std::vector<hipGraphNode_t>& dep = r->tails[s];
    hipGraphNode_t node = nullptr;
    hipError_t e = hipGraphAddKernelNode(&node, r->graph, dep.empty() ? nullptr : dep.data(), dep.size(), &kp);
    if (e == hipSuccess && !node) e = hipErrorInvalidValue;
    if (e != hipSuccess) {
        r->err = e;
        return e;
    }
    r->args.push_back(std::move(blk));
    dep.assign(1, node);
    ++r->launches;
    return hipSuccess;
}

// hipEventRecord / hipStreamWaitEvent of a solve's own fork and join events: dependency
// edges while a recorder is active.
hipError_t rec_event_record(hipEvent_t ev, hipStream_t s);
hipError_t rec_stream_wait(hipStream_t s, hipEvent_t ev);

// ------------------------------------------------------------------ constants of the operator
// Level 0 uses the exact lattice Green's function.  Levels >= 1 use it too when the
// interval nodes fall on the lattice (integer node spacing) and max|x_i| < kLatticeRadius;
// everywhere else the far kernel is the asymptotic expansion with kFarTerms terms.
constexpr int kLatticeRadius = 32;
constexpr int kFarTerms = 8;

// Grid of a persistent kernel over ntiles tiles (a workgroup takes tiles blockIdx.x,
// blockIdx.x + gridDim.x, ...): as many workgroups as are resident at once when the
// kernel's occupancy is at most max_per_cu workgroups per CU, where a workgroup's own
// latency would otherwise idle its CU; else one workgroup per tile.
template <typename K>
int64_t persistent_grid(K kernel, int nt, int64_t ntiles, int max_per_cu) {
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int64_t> cache;  // (device, kernel) -> resident workgroups
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    const auto key = std::make_pair(dev, reinterpret_cast<const void*>(kernel));
    int64_t resident = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            resident = it->second;
        } else {
            int per_cu = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess || per_cu < 1)
                per_cu = 1;
            if (dev < 0 ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
                cus = 256;
            resident = per_cu <= max_per_cu ? (int64_t)per_cu * cus : 0;  // 0: one workgroup per tile
            cache[key] = resident;
        }
    }
    return resident > 0 ? std::min(ntiles, resident) : ntiles;
}

// ------------------------------------------------------------------ launchers (device code)
// out: chunk-major spectra of nout items, of which the first nbatch are written (nout = 0:
// nbatch + 1, the last a zero sentinel that is not written)
// nt: threads per workgroup variant (0 = default; tunable for level-0 tiles)
template <typename T>
// scratch: HBM intermediate for the two-phase tiles (m = 17): nbatch * m * 2m * (m + 1)
// complex values of 16 bytes (two_phase_scratch_bytes); unused otherwise
hipError_t launch_pad_fft(int m, const T* in, cplx<T>* out, int64_t nbatch, hipStream_t s, int nt = 0,
                          int64_t nout = 0, void* scratch = nullptr);
// out_map: output tile of each transformed item (NULL = the item's own index); opitch:
// edge of the output tiles (0 = m; larger pads the m^3 results with zero planes, m = 16)
template <typename Tin, typename A, typename Tout>
hipError_t launch_ifft_trunc(int m, const cplx<Tin>* in, Tout* out, int64_t nbatch, hipStream_t s, int nt = 0,
                             const int32_t* out_map = nullptr, void* scratch = nullptr, int opitch = 0);
// Forward transforms of several levels in one launch (tiles of m <= 10; nout as above,
// 0 = nbatch + 1; at most kMaxFarSegs levels, each with nbatch > 0).
template <typename T>
struct FwdLevel {
    const T* in;
    cplx<T>* out;
    int64_t nbatch, nout;
};
template <typename T>
hipError_t launch_pad_fft_levels(int m, const FwdLevel<T>* lv, int nlev, hipStream_t s);
// The same for several levels' spectra in one launch (tiles of m <= 10, outputs in item
// order, at most kMaxFarSegs levels, each with nbatch > 0).
template <typename Tin, typename Tout>
struct InvLevel {
    const cplx<Tin>* in;
    Tout* out;
    int64_t nbatch;
};
template <typename Tin, typename A, typename Tout>
hipError_t launch_ifft_trunc_levels(int m, const InvLevel<Tin, Tout>* lv, int nlev, hipStream_t s);

// Far-field node values of the down pass: double on the FP64 path, float-float on the
// FP32 path (8 bytes either way).
template <typename T> struct FarAcc;
template <> struct FarAcc<double> { using type = double; };
template <> struct FarAcc<float> { using type = ff32; };

// Source spectra (fhat) arrays hold nitems + 1 items per frequency chunk; the last is a zero
// sentinel that inactive neighbours point to.  Field spectra (uhat) hold nitems items.
// Level 0 over groups of 2x2x2 target blocks (tgt8) with their 4^3 source neighbourhood (src64).
// Sources and targets are numbered separately: fhat holds nsrc + 1 items (sentinel nsrc),
// uhat ntgt items.
// prefetch: 1 = the next source slab's loads are issued before the current slab is used.
template <typename T>
hipError_t launch_prod_near(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* tgt8, const int32_t* src64,
                            cplx<T>* uhat, int64_t ngroups, int64_t nsrc, int64_t ntgt, int S, int waves,
                            int prefetch, hipStream_t s, const SpecSym& sym = SpecSym{});
// sym: a reduced kernel table (khat then holds sym.ncls spectra) must match the spectrum
// size S = M^2 (M/2 + 1) and hold at most 65536 spectra
inline bool sym_fits(const SpecSym& y, int S) {
    return !y.info || (y.M > 0 && y.ncls > 0 && y.ncls <= 65536 && S == y.M * y.M * (y.M / 2 + 1));
}
// Levels >= 1 below the top: over parents (child8 and the 216 candidate sources src216 of
// each parent), offsets radius 3.
// waves: parent groups per workgroup (1, 2, 4); cpl: children accumulated per lane (8, 4, 2,
// 1); 0 = chosen from the level's size.
template <typename T>
// fhat holds nsrc + 1 items (sentinel nsrc), uhat nitems items; nsrc = nitems unless the
// level reads another level's spectra (level 1 of the lattice scheme reads the blocks').
hipError_t launch_prod_far_sib(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* child8,
                               const int32_t* src216, cplx<T>* uhat, int64_t nparents, int64_t nitems, int64_t nsrc,
                               int S, int waves, int cpl, hipStream_t s, const SpecSym& sym = SpecSym{});
// The same over several levels in one launch, each with its own spectrum size S (at most
// kMaxFarSegs levels, each with nparents > 0, in the order given).
constexpr int kMaxFarSegs = 8;
template <typename T>
struct FarLevel {
    const cplx<T>* fhat;
    const cplx<T>* khat;
    const int32_t* child8;
    const int32_t* src216;
    cplx<T>* uhat;
    int64_t nparents, nitems, nsrc;
    int S;
    SpecSym sym;  // reduced kernel spectra, or none
};
template <typename T>
hipError_t launch_prod_far_sib_levels(const FarLevel<T>* lv, int nlev, int waves, int cpl, hipStream_t s);
// Targets tgt[0..ntgt) from CSR lists (the top level of a truncated tree); fhat holds
// nsrc + 1 items (nsrc < 0: nitems).
template <typename T>
hipError_t launch_prod_far(const cplx<T>* fhat, const cplx<T>* khat, const int32_t* ptr, const int32_t* src,
                           const int32_t* off, const int32_t* tgt, cplx<T>* uhat, int64_t ntgt, int64_t nitems,
                           int noff, int S, hipStream_t s, int64_t nsrc = -1, const SpecSym& sym = SpecSym{});

// Kernel variants picked per plan (by the autotuner, or defaults).
struct TuneConfig {
    int fft0_threads = 0;  // 0 = default per tile size, else 128 / 256 / 512
    int near_waves = 4;    // waves per workgroup of the level-0 Prod kernel: 2, 4, 8
    int near_prefetch = 0; // that kernel's source loads half a z slab ahead: 0, 1 (by plan size)
    int far_waves = 0;     // parent groups per workgroup of the level >= 1 Prod kernel: 1, 2, 4, 0 = by level size
    int far_children = 0;  // children per lane of that kernel: 8, 4, 2, 1, or 0 = by level size
    int overlap = 0;       // far-field chain on a second stream: 1 = yes, 2 = no, 0 = default (yes)
};

// Reg block -> level-1 interval: out[b] = (A x A x A) f[b], A is p x n (row-major)
template <typename T>
hipError_t launch_reg_block(const T* f, const double* A, T* out, int64_t nb, int n, int p, hipStream_t s);
// Reg children -> parent: out[J] = sum_c (C_cz x C_cy x C_cx) in[child_c(J)]
template <typename T>
// scratch: p = 17 only, nparent * 8 * p^3 values of T (the children's partial sums)
hipError_t launch_reg_up(const T* in, const int32_t* child8, const double* C01, T* out, int64_t nparent, int p,
                         hipStream_t s, void* scratch = nullptr);
// Level-1 node values of the lattice scheme: out[b] (p^3) = f[b] (n^3) padded with zeros
template <typename T>
hipError_t launch_pad_copy(const T* f, T* out, int64_t nb, int n, int p, hipStream_t s);
// Interp parent -> its children, accumulate: io[child8[J][c]] += (C_c^T x C_c^T x C_c^T) par[J]
template <typename U>
hipError_t launch_interp_down(const U* par, const int32_t* child8, const double* C01, U* io, int64_t nparent,
                              int p, hipStream_t s);
// Final: u[b] = vnear[b] + (A^T x A^T x A^T) ut[q(b)], accumulated in FP64 (u may alias
// vnear); q(b) = l1map[b] (the level-1 interval of evaluation block b), or b when l1map is
// NULL; vnear[b] is taken as 0 (and not read) where near_flag[b] == 0 (NULL: every block)
template <typename T, typename U>
hipError_t launch_final(const T* vnear, const U* ut, const double* A, T* u, int64_t nb, int n, int p,
                        hipStream_t s, const int32_t* l1map = nullptr, const int32_t* near_flag = nullptr);

// ------------------------------------------------------------------ kernel spectra
struct SpectraKey {
    int n, p, level;   // level 0 = near field
    int radius;        // offsets D in [-radius, radius]^3, id = (Dx+R) + (2R+1)((Dy+R) + (2R+1)(Dz+R))
    int prec;          // 0 = f64, 1 = f32
    int m = 0;         // tile edge (0: n at level 0, p above; n at level 1 of the lattice scheme)
    int sym = 0;       // 1 = symmetry-reduced table (one spectrum per class of offsets)
    double kappa = 0;  // screening of the operator L - kappa (0: the Laplace LGF)
    bool operator<(const SpectraKey& o) const;
};

struct SpectraEntry {
    SpectraKey key;
    int M = 0, S = 0, noff = 0;
    void* dev = nullptr;  // noff x S complex of the plan precision, chunk-major (spec_at), scaled by 1/M^3;
                          // reduced tables: ncls x S, with the per-offset descriptions in dev_info
    uint32_t* dev_info = nullptr;
    SpecSym sym;          // view of the reduced table (sym.info == nullptr: full table)
    int64_t bytes = 0;
    ~SpectraEntry();
};

// Get or build the spectra (FP64 generation; rounded to FP32 for prec 1).
std::shared_ptr<SpectraEntry> get_spectra(const SpectraKey& key, hipStream_t s, std::string& err);
int64_t spectra_bytes_total();
void spectra_trim();
// Table kind for plans created afterwards (process-wide): 0 = one spectrum per offset,
// 1 = symmetry-reduced.
void spectra_set_mode(int mode);
int spectra_mode();
// The calling thread's own mode (-1: follow the process-wide one); the request server's
// dispatcher keeps the mode the server was created with.
void spectra_set_thread_mode(int mode);
// Classes of the offsets D in [-R, R]^3 under the 48 signed axis permutations, and each
// offset's description (the layout of SpecSym::info); returns the number of classes.
int spectra_classes(int R, std::vector<uint32_t>& info, std::vector<int32_t>& rep_offset);

// LGF table [R][R][R] (full octant) on the device, FP64, cached per R.
const double* green_table_device(int R, hipStream_t s, std::string& err);
// LGF of the screened operator L - kappa (kappa >= kKappaMin) at lattice spacing h:
// T[(a*R + b)*R + c] = G_kappa(h a, h b, h c), 0 <= a, b, c < R; device, FP64, cached.
constexpr double kKappaMin = 1e-3;
const double* screened_table_device(int R, int h, double kappa, hipStream_t s, std::string& err);
// far kernel A^q at device points (FP64): out[i] = A^q(pts[i])
hipError_t far_kernel_device(const double* pts, int64_t npts, double* out, hipStream_t s, std::string& err);
// The same at HOST points into HOST out, staged through the library's static device array
// (no device allocation); npts <= LGF_FAR_KERNEL_NOALLOC_MAX_POINTS.  Synchronous.
hipError_t far_kernel_noalloc(const double* pts, int64_t npts, double* out, std::string& err);

// ------------------------------------------------------------------ memory accounting
bool budget_reserve(int64_t bytes);
void budget_release(int64_t bytes);
int64_t budget_in_use();
void budget_set(int64_t bytes);

// Workspace bytes a plan of this layout would own (host-only work: builds the lists).
lgf_status plan_estimate(const int32_t* ijk, int64_t nblocks, int n, int p, int levels, lgf_precision prec,
                         int64_t* bytes);

}  // namespace lgfdev
