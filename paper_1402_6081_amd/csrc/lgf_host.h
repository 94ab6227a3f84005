// Host description of a plan, free of device code: the octree of intervals and its lists
// (Sec. 3.1: RegSupp, IntrpSupp, InflList), the 1D Lagrange basis (Sec. 2.5), unions of
// independent layouts, workspace sizes, and the calling thread's error message.  The
// library compiles it with the rest; the host checks also build it alone, with the address
// and undefined-behaviour sanitizers.
//
// Tree conventions: block coordinates are shifted so the bounding-box minimum is 0; the
// level-1 interval of block B has index B and the parent of interval I is floor(I / 2).
// Interval I at level l spans [I s_l, (I+1) s_l]^3, s_l = n 2^(l-1), with nodes I s_l + k h_l,
// h_l = s_l / (p - 1), k in [0, p)^3.  Lists: level 0 near neighbours |Q-P|_inf <= 1; level
// l < L: children of the parent's neighbours with |Q-P|_inf >= 2; top level L: every
// interval with |Q-P|_inf >= 2.
#ifndef LGF_HOST_H_
#define LGF_HOST_H_

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lgf.h"

namespace lgfdev {

constexpr int kMaxLevels = 16;
constexpr int kNmax = 10;  // most nodes one interpolation stencil uses (the paper's n_max)

// Every spectrum array is stored in chunks of 64 frequencies (see spec_at); the per-item
// half-spectrum size is padded to a whole number of chunks.
constexpr int kSpecChunk = 64;
constexpr int spec_padded(int S) { return (S + kSpecChunk - 1) / kSpecChunk * kSpecChunk; }

// Tiles of 17 nodes take the two-phase transforms, whose HBM intermediate holds
// nbatch * m * 2m * (m + 1) complex values of 16 bytes.
inline bool two_phase_tile(int m) { return m == 17; }
inline int64_t two_phase_scratch_bytes(int m, int64_t nbatch) {
    return two_phase_tile(m) ? nbatch * (int64_t)m * (2 * m) * (m + 1) * 16 : 0;
}

// Block edges n the transforms take (padded length 2n), and the node counts p allowed with
// them: 2..10 (every stencil uses all p nodes), or p = n + 1 > n_max for n = 12 and 16 (the
// paper's scheme n_I = n + 1 with stencils of the n_max closest nodes).
inline bool block_edge_ok(int n) { return n == 4 || n == 6 || n == 8 || n == 12 || n == 16; }
inline bool nodes_ok(int n, int p) { return p >= 2 && (p <= kNmax || ((n == 12 || n == 16) && p == n + 1)); }

// The calling thread's lgf_last_error message.
std::string& err_text();
inline void set_last_error(const std::string& msg) { err_text() = msg; }
inline lgf_status fail(lgf_status st, const std::string& msg) {
    err_text() = msg;
    return st;
}

inline uint64_t pack(int64_t x, int64_t y, int64_t z) {
    return (uint64_t)x | ((uint64_t)y << 21) | ((uint64_t)z << 42);
}

// Lagrange basis of node k among the nodes 0..p-1 at t (Sec. 2.5).  With more than
// kNmax nodes only the kNmax consecutive nodes closest to t are used (hybrid p/h
// refinement): the window starts at ceil(t - kNmax/2), ties going to the lower window,
// clamped to the interval, and nodes outside it get 0.
long double lagrange(int p, int k, long double t);

struct HostLevel {
    int64_t nint = 0;
    int64_t nsrc_int = 0;         // intervals holding a source (the spectra the lists read)
    std::vector<int32_t> coords;  // [nint][3] (single layouts only; empty in unions)
    std::vector<int32_t> child8;  // [nint][8] children at level l-1 (levels >= 2)
    std::vector<int32_t> src216;  // [nint][216] children of the 27 neighbours, sentinel = N_{l-1}
    int64_t sib_pairs = 0;        // interaction-list entries of targets served through parents
    // top level of a truncated tree: explicit lists over a target subset
    std::vector<int32_t> csr_tgt, csr_ptr{0}, csr_src;
    std::vector<std::array<int32_t, 3>> csr_D;
    bool zero_uhat = false;  // some targets are served by neither list kind (unions)
    int64_t pairs() const { return sib_pairs + (int64_t)csr_src.size(); }
};

struct HostPlan {
    int n = 0, p = 0, L = 0, Ltop = 0;
    // the lattice scheme with local stencils (p = n + 1 > n_max): level-1 nodes are the
    // blocks' grid points, and level 1 works on the blocks' own spectra (tiles of n)
    bool lat1 = false;
    int64_t nb = 0, near_pairs = 0, ngroups0 = 0;
    int64_t nsrc = 0, neval = 0;              // source / evaluation blocks (both nb unless split)
    std::vector<int32_t> eval_l1;             // split sets: level-1 interval of each evaluation block
    int64_t ntgt0 = 0;                        // level-0 targets transformed (near-active blocks)
    std::vector<int32_t> near_out;            // split sets: evaluation block of each level-0 target
    std::vector<int32_t> near_flag;           // split sets: 1 if the evaluation block has a near field
    std::vector<int32_t> g0_tgt8, g0_src64;  // targets: evaluation numbering; sources: sentinel = nsrc
    std::vector<HostLevel> lv;               // index 0 unused, 1..L
    std::vector<int64_t> solve_offsets{0};   // block offsets of the layouts of a batch
    // levels >= 1: does an interval hold a source / an evaluation block below it (index = level)
    std::vector<std::vector<char>> has_src, has_eval;
};


// Source blocks ijk[nblocks] and evaluation blocks (Eq. bconv).  With eval_ijk == NULL the
// two sets are the same blocks.  Otherwise the levels >= 1 are built over the union of the
// two sets, sources first (the union index of source block i is i), then the evaluation
// blocks that are not sources.  An interval with no source below it carries a zero field: the
// source lists name the zero sentinel instead, so it costs no spectrum reads.  An interval
// with no evaluation block below it is never interpolated to a block, and the list sizes
// reported count only pairs with an evaluation target (the lists of the method).  The level-0
// groups hold evaluation blocks (numbered as given) and their sources (numbered as given).
lgf_status build_host(const int32_t* ijk, int64_t nblocks, int n, int p, int levels, HostPlan& H,
                      const int32_t* eval_ijk = nullptr, int64_t neval = 0);

// Every list index within its array's range; LGF_ERR_LAYOUT otherwise.
lgf_status check_host(const HostPlan& H);

// Union of independent layouts: every index is offset by the items of the earlier
// layouts; sentinels map to the union's sentinel; lists never cross layouts.
HostPlan concat(const std::vector<HostPlan>& parts);

// HBM intermediate of the two-phase transforms and of the 17-node Reg up.
int64_t scratch_need(const HostPlan& H);

// Device bytes of a plan's workspace (lists, matrices, node values and spectra of every
// level it solves on); the shared kernel spectra are not included.
int64_t workspace_need(const HostPlan& H, lgf_precision prec);

}  // namespace lgfdev

#endif  // LGF_HOST_H_
