// Host description of a plan: tree, lists, Lagrange basis, unions and workspace sizes (see
// lgf_host.h).  Plain C++, no device code.
#include "lgf_host.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace lgfdev {

std::string& err_text() {
    thread_local std::string t;
    return t;
}

// Lagrange basis of node k among the nodes 0..p-1 at t (Sec. 2.5).  With more than
// kNmax nodes only the kNmax consecutive nodes closest to t are used (hybrid p/h
// refinement): the window starts at ceil(t - kNmax/2), ties going to the lower window,
// clamped to the interval, and nodes outside it get 0.
long double lagrange(int p, int k, long double t) {
    int lo = 0, hi = p;
    if (p > kNmax) {
        lo = (int)std::ceil(t - kNmax / 2.0L);
        lo = std::min(std::max(lo, 0), p - kNmax);
        hi = lo + kNmax;
    }
    if (k < lo || k >= hi) return 0.0L;
    long double v = 1.0L;
    for (int j = lo; j < hi; ++j)
        if (j != k) v *= (t - j) / (long double)(k - j);
    return v;
}

// Source blocks ijk[nblocks] and evaluation blocks (Eq. bconv).  With eval_ijk == NULL the
// two sets are the same blocks.  Otherwise the levels >= 1 are built over the union of the
// two sets, sources first (the union index of source block i is i), then the evaluation
// blocks that are not sources.  An interval with no source below it carries a zero field: the
// source lists name the zero sentinel instead, so it costs no spectrum reads.  An interval
// with no evaluation block below it is never interpolated to a block, and the list sizes
// reported count only pairs with an evaluation target (the lists of the method).  The level-0
// groups hold evaluation blocks (numbered as given) and their sources (numbered as given).
lgf_status build_host(const int32_t* ijk, int64_t nblocks, int n, int p, int levels, HostPlan& H,
                      const int32_t* eval_ijk, int64_t neval) {
    const bool split = eval_ijk != nullptr;
    if (!split) {
        eval_ijk = ijk;
        neval = nblocks;
    }
    H.n = n;
    H.p = p;
    H.lat1 = p == n + 1 && p > kNmax;
    H.nsrc = nblocks;
    H.neval = neval;
    int64_t lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, hi[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    auto span = [&](const int32_t* c, int64_t m) {
        for (int64_t b = 0; b < m; ++b)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min<int64_t>(lo[d], c[3 * b + d]);
                hi[d] = std::max<int64_t>(hi[d], c[3 * b + d]);
            }
    };
    span(ijk, nblocks);
    if (split) span(eval_ijk, neval);
    int64_t ext = 1;
    for (int d = 0; d < 3; ++d) {
        if (hi[d] - lo[d] >= (1 << 20)) return fail(LGF_ERR_LAYOUT, "layout spans more than 2^20 blocks");
        ext = std::max<int64_t>(ext, hi[d] - lo[d] + 1);
    }
    const int64_t cap = nblocks + (split ? neval : 0);
    std::vector<int32_t> blocks;  // the union, shifted so the minimum is 0
    blocks.reserve(3 * cap);
    std::unordered_map<uint64_t, int32_t> idx0;  // union index of a block
    idx0.reserve(cap * 2);
    for (int64_t b = 0; b < nblocks; ++b) {
        int32_t c[3];
        for (int d = 0; d < 3; ++d) c[d] = (int32_t)(ijk[3 * b + d] - lo[d]);
        if (!idx0.emplace(pack(c[0], c[1], c[2]), (int32_t)b).second)
            return fail(LGF_ERR_LAYOUT, split ? "duplicate source block" : "duplicate block in layout");
        blocks.insert(blocks.end(), c, c + 3);
    }
    std::vector<int32_t> ecoords;  // evaluation blocks, shifted (split sets only)
    if (split) {
        std::unordered_set<uint64_t> seen;
        seen.reserve(neval * 2);
        ecoords.resize(3 * neval);
        H.eval_l1.resize(neval);
        for (int64_t j = 0; j < neval; ++j) {
            int32_t* c = &ecoords[3 * j];
            for (int d = 0; d < 3; ++d) c[d] = (int32_t)(eval_ijk[3 * j + d] - lo[d]);
            const uint64_t key = pack(c[0], c[1], c[2]);
            if (!seen.insert(key).second) return fail(LGF_ERR_LAYOUT, "duplicate evaluation block");
            auto it = idx0.find(key);
            int32_t u;
            if (it == idx0.end()) {
                u = (int32_t)(blocks.size() / 3);
                idx0.emplace(key, u);
                blocks.insert(blocks.end(), c, c + 3);
            } else {
                u = it->second;
            }
            H.eval_l1[j] = u;
        }
    }
    const int64_t nu = (int64_t)blocks.size() / 3;
    H.nb = nu;
    H.solve_offsets = {0, neval};
    int full = 1;
    while ((int64_t(1) << (full - 1)) < ext) ++full;
    H.L = levels <= 0 ? full : std::min(levels, full);
    if (H.L >= kMaxLevels) return fail(LGF_ERR_LAYOUT, "tree deeper than supported");

    // ---- levels: coordinates, parents, children, and which intervals hold sources /
    //      evaluation blocks
    H.lv.assign(H.L + 1, HostLevel());
    H.has_src.assign(H.L + 1, std::vector<char>());
    H.has_eval.assign(H.L + 1, std::vector<char>());
    std::vector<std::unordered_map<uint64_t, int32_t>> idx(H.L + 2);
    H.lv[1].nint = nu;
    H.lv[1].coords = blocks;
    idx[1] = idx0;
    H.has_src[1].assign(nu, 0);
    H.has_eval[1].assign(nu, split ? 0 : 1);
    for (int64_t i = 0; i < nblocks; ++i) H.has_src[1][i] = 1;
    for (int32_t u : H.eval_l1) H.has_eval[1][u] = 1;
    for (int l = 1; l < H.L; ++l) {
        HostLevel& C = H.lv[l];
        HostLevel& P = H.lv[l + 1];
        std::vector<int32_t> parent(C.nint), cpos(C.nint);
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
            parent[i] = j;
            cpos[i] = (x & 1) | ((y & 1) << 1) | ((z & 1) << 2);
        }
        P.child8.assign(8 * P.nint, -1);
        H.has_src[l + 1].assign(P.nint, 0);
        H.has_eval[l + 1].assign(P.nint, 0);
        for (int64_t i = 0; i < C.nint; ++i) {
            P.child8[8 * parent[i] + cpos[i]] = (int32_t)i;
            H.has_src[l + 1][parent[i]] |= H.has_src[l][i];
            H.has_eval[l + 1][parent[i]] |= H.has_eval[l][i];
        }
    }
    // ---- levels >= 2: the 216 candidate sources of each parent (children of its neighbours);
    //      the interaction-list size of every child follows from them
    for (int l = 2; l <= H.L; ++l) {
        HostLevel& Lv = H.lv[l];
        const HostLevel& Ch = H.lv[l - 1];
        // the zero sentinel of the spectra the lists index: level 1 of the lattice scheme
        // reads the level-0 source spectra (nsrc items and the sentinel)
        const int32_t sentinel = (int32_t)(l == 2 && H.lat1 ? H.nsrc : Ch.nint);
        Lv.src216.assign(216 * Lv.nint, sentinel);
        int64_t pairs = 0;
        for (int64_t i = 0; i < Lv.nint; ++i) {
            for (int e = 0; e < 27; ++e) {
                const int64_t jx = Lv.coords[3 * i] + e % 3 - 1, jy = Lv.coords[3 * i + 1] + (e / 3) % 3 - 1,
                              jz = Lv.coords[3 * i + 2] + e / 9 - 1;
                if (jx < 0 || jy < 0 || jz < 0) continue;
                auto it = idx[l].find(pack(jx, jy, jz));
                if (it == idx[l].end()) continue;
                for (int cs = 0; cs < 8; ++cs) {
                    const int32_t q = Lv.child8[8 * it->second + cs];
                    if (q >= 0 && H.has_src[l - 1][q]) Lv.src216[216 * i + 8 * e + cs] = q;
                }
            }
            for (int c = 0; c < 8; ++c) {
                const int32_t t = Lv.child8[8 * i + c];
                if (t < 0 || !H.has_eval[l - 1][t]) continue;
                for (int s = 0; s < 216; ++s) {
                    const int32_t q = Lv.src216[216 * i + s];
                    if (q == sentinel) continue;
                    const int32_t* P = &Ch.coords[3 * t];
                    const int32_t* Q = &Ch.coords[3 * q];
                    const int dinf =
                        std::max(std::abs(P[0] - Q[0]), std::max(std::abs(P[1] - Q[1]), std::abs(P[2] - Q[2])));
                    if (dinf >= 2) ++pairs;
                }
            }
        }
        H.lv[l - 1].sib_pairs = pairs;
    }
    // ---- top level: every non-adjacent interval (non-empty only below the full depth); a
    //      target without evaluation blocks keeps an empty list (its field is written as 0)
    {
        HostLevel& T = H.lv[H.L];
        for (int64_t i = 0; i < T.nint; ++i) {
            const int32_t* P = &T.coords[3 * i];
            T.csr_tgt.push_back((int32_t)i);
            for (int64_t q = 0; q < T.nint && H.has_eval[H.L][i]; ++q) {
                if (!H.has_src[H.L][q]) continue;
                const int32_t* Q = &T.coords[3 * q];
                std::array<int32_t, 3> D{P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
                if (std::max(std::abs(D[0]), std::max(std::abs(D[1]), std::abs(D[2]))) < 2) continue;
                T.csr_src.push_back((int32_t)q);
                T.csr_D.push_back(D);
            }
            T.csr_ptr.push_back((int32_t)T.csr_src.size());
        }
        if (T.csr_src.empty()) {
            T.csr_tgt.clear();
            T.csr_ptr = {0};
        }
    }
    for (int l = 1; l <= H.L; ++l) {
        if (H.lv[l].pairs() > 0) H.Ltop = l;
        for (char c : H.has_src[l]) H.lv[l].nsrc_int += c;
    }

    // ---- level 0: near pairs (evaluation target, source) and 2x2x2 target groups with
    //      their 4^3 source neighbourhood.  With separate sets and a far field, evaluation
    //      blocks with no source among their 27 neighbours have a zero near field: they get
    //      no level-0 target (the final pass adds the far field alone), so the level-0
    //      targets are the near-active blocks, numbered in evaluation order.
    auto source_at = [&](int64_t qx, int64_t qy, int64_t qz) -> int32_t {
        if (qx < 0 || qy < 0 || qz < 0) return -1;
        auto jt = idx0.find(pack(qx, qy, qz));
        return (jt != idx0.end() && jt->second < nblocks) ? jt->second : -1;
    };
    const int32_t* E = split ? ecoords.data() : blocks.data();
    const bool trim = split && H.Ltop >= 1;
    std::vector<int32_t> act(neval, -1);
    for (int64_t b = 0; b < neval; ++b) {
        const int32_t* P = &E[3 * b];
        int cnt = 0;
        for (int d = 0; d < 27; ++d)
            if (source_at(P[0] - (d % 3 - 1), P[1] - ((d / 3) % 3 - 1), P[2] - (d / 9 - 1)) >= 0) ++cnt;
        H.near_pairs += cnt;
        if (!trim || cnt > 0) {
            act[b] = (int32_t)H.ntgt0++;
            if (trim) H.near_out.push_back((int32_t)b);
        }
    }
    if (trim && H.ntgt0 == neval) {
        H.near_out.clear();  // every evaluation block is near-active: identity
    } else if (trim) {
        H.near_flag.assign(neval, 0);
        for (int64_t b = 0; b < neval; ++b) H.near_flag[b] = act[b] >= 0;
    }
    std::unordered_map<uint64_t, int32_t> gidx;
    for (int64_t b = 0; b < neval; ++b) {
        if (act[b] < 0) continue;
        const int32_t* P = &E[3 * b];
        const uint64_t key = pack(P[0] >> 1, P[1] >> 1, P[2] >> 1);
        auto it = gidx.find(key);
        int32_t g;
        if (it == gidx.end()) {
            g = (int32_t)H.ngroups0++;
            gidx.emplace(key, g);
            H.g0_tgt8.resize(8 * H.ngroups0, -1);
            H.g0_src64.resize(64 * H.ngroups0, (int32_t)nblocks);
            for (int sidx = 0; sidx < 64; ++sidx) {
                const int32_t q = source_at(2 * (int64_t)(P[0] >> 1) + (sidx & 3) - 1,
                                            2 * (int64_t)(P[1] >> 1) + ((sidx >> 2) & 3) - 1,
                                            2 * (int64_t)(P[2] >> 1) + (sidx >> 4) - 1);
                if (q >= 0) H.g0_src64[64 * g + sidx] = q;
            }
        } else {
            g = it->second;
        }
        H.g0_tgt8[8 * g + ((P[0] & 1) | ((P[1] & 1) << 1) | ((P[2] & 1) << 2))] = act[b];
    }
    return LGF_OK;
}

// Every index a kernel will follow lies inside the buffer it addresses (checked on the host
// before upload): level-0 targets < ntgt0, sources <= nsrc (the sentinel), output maps inside
// the caller's u and the level-1 fields, children and candidate sources inside their level.
lgf_status check_host(const HostPlan& H) {
    auto within = [](const std::vector<int32_t>& v, int64_t lo, int64_t hi) {
        for (int32_t x : v)
            if (x < lo || x > hi) return false;
        return true;
    };
    bool ok = within(H.g0_tgt8, -1, H.ntgt0 - 1) && within(H.g0_src64, 0, H.nsrc) &&
              within(H.eval_l1, 0, H.nb - 1) && within(H.near_out, 0, H.neval - 1) &&
              (H.near_out.empty() || (int64_t)H.near_out.size() == H.ntgt0) &&
              (H.near_flag.empty() || (int64_t)H.near_flag.size() == H.neval) &&
              (int64_t)H.g0_tgt8.size() == 8 * H.ngroups0 && (int64_t)H.g0_src64.size() == 64 * H.ngroups0 &&
              H.ntgt0 <= H.neval && H.nsrc <= H.nb && (H.eval_l1.empty() || (int64_t)H.eval_l1.size() == H.neval);
    for (int l = 2; ok && l <= H.L && l < (int)H.lv.size(); ++l) {
        const HostLevel& Lv = H.lv[l];
        const int64_t nc = H.lv[l - 1].nint;
        // level 1 of the lattice scheme reads the level-0 source spectra (nsrc and the sentinel)
        const int64_t ns = l == 2 && H.lat1 ? H.nsrc : nc;
        ok = within(Lv.child8, -1, nc - 1) && within(Lv.src216, 0, ns) &&
             (Lv.src216.empty() || (int64_t)Lv.src216.size() == 216 * Lv.nint);
    }
    for (int l = 1; ok && l <= H.L && l < (int)H.lv.size(); ++l) {
        const HostLevel& Lv = H.lv[l];
        const int64_t ns = l == 1 && H.lat1 ? H.nsrc : Lv.nint;
        ok = within(Lv.csr_tgt, 0, Lv.nint - 1) && within(Lv.csr_src, 0, ns - 1) &&
             Lv.csr_ptr.size() == Lv.csr_tgt.size() + 1 && (int64_t)Lv.csr_ptr.back() == (int64_t)Lv.csr_src.size();
    }
    return ok ? LGF_OK : fail(LGF_ERR_LAYOUT, "internal error: plan list index out of range");
}

// Union of independent layouts: every index is offset by the items of the earlier
// layouts; sentinels map to the union's sentinel; lists never cross layouts.
HostPlan concat(const std::vector<HostPlan>& parts) {
    HostPlan U;
    U.n = parts[0].n;
    U.p = parts[0].p;
    U.lat1 = parts[0].lat1;
    for (const auto& P : parts) {
        U.L = std::max(U.L, P.L);
        U.Ltop = std::max(U.Ltop, P.Ltop);
    }
    U.lv.assign(U.L + 1, HostLevel());
    for (const auto& P : parts) {
        U.nb += P.nb;
        U.nsrc += P.nsrc;  // parts have equal source and evaluation sets
        U.neval += P.neval;
        U.ntgt0 += P.ntgt0;
        U.ngroups0 += P.ngroups0;
        U.near_pairs += P.near_pairs;
        for (int l = 1; l <= P.L; ++l) {
            U.lv[l].nint += P.lv[l].nint;
            U.lv[l].nsrc_int += P.lv[l].nsrc_int;
        }
    }
    U.solve_offsets = {0};
    std::vector<int64_t> off(U.L + 1, 0);  // running item offset per level (level 1 = blocks)
    for (const auto& P : parts) {
        const int64_t ob = off[1];
        for (int32_t t : P.g0_tgt8) U.g0_tgt8.push_back(t < 0 ? -1 : (int32_t)(t + ob));
        for (int32_t q : P.g0_src64) U.g0_src64.push_back(q == (int32_t)P.nsrc ? (int32_t)U.nsrc : (int32_t)(q + ob));
        for (int l = 1; l <= P.L; ++l) {
            const HostLevel& A = P.lv[l];
            HostLevel& B = U.lv[l];
            B.sib_pairs += A.sib_pairs;
            if (l >= 2) {
                const int64_t oc = off[l - 1];
                const int32_t sent_in = (int32_t)P.lv[l - 1].nint, sent_out = (int32_t)U.lv[l - 1].nint;
                for (int32_t c : A.child8) B.child8.push_back(c < 0 ? -1 : (int32_t)(c + oc));
                for (int32_t q : A.src216) B.src216.push_back(q == sent_in ? sent_out : (int32_t)(q + oc));
            }
            const int64_t ol = off[l];
            for (int32_t t : A.csr_tgt) B.csr_tgt.push_back((int32_t)(t + ol));
            for (size_t k = 1; k < A.csr_ptr.size(); ++k)
                B.csr_ptr.push_back((int32_t)(B.csr_src.size() + A.csr_ptr[k]));
            for (int32_t q : A.csr_src) B.csr_src.push_back((int32_t)(q + ol));
            for (const auto& D : A.csr_D) B.csr_D.push_back(D);
            // a layout's top level with an empty list gets no Prod: clear its targets' fields
            if (l == P.L && A.csr_src.empty()) B.zero_uhat = true;
        }
        for (int l = 1; l <= P.L; ++l) off[l] += P.lv[l].nint;
        U.solve_offsets.push_back(off[1]);
    }
    return U;
}

// HBM intermediate of the two-phase transforms (levels >= 2 of a tile that does not fit one
// workgroup's LDS); the levels run one after another on one stream and share it.
int64_t scratch_need(const HostPlan& H) {
    int64_t nmax = 0, pmax = 0;
    for (int l = 1; l <= H.Ltop; ++l)
        if (H.lv[l].pairs() > 0 && !(l == 1 && H.lat1)) nmax = std::max(nmax, H.lv[l].nint);
    for (int l = 2; l <= H.Ltop; ++l) pmax = std::max(pmax, H.lv[l].nint);  // Reg up: children's partials
    const int64_t p3 = (int64_t)H.p * H.p * H.p;
    const int64_t reg = H.p > kNmax ? pmax * 8 * p3 * 8 : 0;  // Reg up of the local-stencil scheme
    return std::max(two_phase_scratch_bytes(H.p, nmax), reg);
}

// Device bytes of a plan's workspace (lists, matrices, node values and spectra of every
// level it solves on); the shared kernel spectra are not included.
int64_t workspace_need(const HostPlan& H, lgf_precision prec) {
    const int n = H.n, p = H.p;
    const int64_t esz = prec == LGF_F64 ? sizeof(double) : sizeof(float);
    const int64_t usz = 8;
    const int64_t S0 = spec_padded(2 * n * 2 * n * (n + 1));
    const int64_t S1 = spec_padded(2 * p * 2 * p * (p + 1));
    const int64_t p3 = (int64_t)p * p * p;
    const int topc = std::min(H.Ltop + 1, H.L);
    int64_t need = H.ngroups0 * 72 * 4 + (p * n + 2 * p * p) * 8 + (H.nsrc + 1 + H.ntgt0) * S0 * 2 * esz +
                   (int64_t)(H.eval_l1.size() + H.near_out.size() + H.near_flag.size()) * 4;
    for (int l = 1; l <= H.Ltop; ++l) {
        const HostLevel& h = H.lv[l];
        need += h.nint * p3 * (esz + usz);
        if (h.pairs() > 0) {
            if (l == 1 && H.lat1)
                need += h.nint * S0 * 2 * esz;  // products only: the sources are the level-0 spectra
            else
                need += (2 * h.nint + 1) * S1 * 2 * esz;
        }
        need += (int64_t)(h.csr_tgt.size() + h.csr_ptr.size() + 2 * h.csr_src.size()) * 4;
    }
    for (int l = 2; l <= topc && H.Ltop >= 1; ++l) need += H.lv[l].nint * 224 * 4;
    return need + scratch_need(H);
}

}  // namespace lgfdev
