// Host checks of the plan's tree and lists (lgf_host.cpp) built on their own, without the
// device code, so that they run under the address and undefined-behaviour sanitizers
// (tests/test_host_sanitized.py).  Reads one case per line from stdin:
//   single n p levels nblocks x y z ...
//   split n p levels nsource neval (source x y z ...) (evaluation x y z ...)
//   batch n p levels count nblocks_1 .. nblocks_count (x y z ... of every layout in turn)
// and prints one line per case: the status, then (if LGF_OK) the union's block count, the
// depth L and top level, near pairs, level-0 groups and targets, source and evaluation
// blocks, the FP64 and FP32 workspace bytes and, per level 1..L, the intervals and the
// far-field pairs.  check_host runs on every plan built.
#include <cstdio>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "lgf_host.h"

using namespace lgfdev;

namespace {

void print(const HostPlan& H) {
    std::printf("0 %lld %d %d %lld %lld %lld %lld %lld %lld %lld", (long long)H.nb, H.L, H.Ltop,
                (long long)H.near_pairs, (long long)H.ngroups0, (long long)H.ntgt0, (long long)H.nsrc,
                (long long)H.neval, (long long)workspace_need(H, LGF_F64), (long long)workspace_need(H, LGF_F32));
    for (int l = 1; l <= H.L; ++l) std::printf(" %lld %lld", (long long)H.lv[l].nint, (long long)H.lv[l].pairs());
    std::printf("\n");
}

std::vector<int32_t> read_blocks(std::istringstream& in, long long nb) {
    std::vector<int32_t> v(3 * nb);
    for (auto& x : v) in >> x;
    return v;
}

}  // namespace

int main() {
    std::string line;
    while (std::getline(std::cin, line)) {
        if (line.empty()) continue;
        std::istringstream in(line);
        std::string kind;
        int n = 0, p = 0, levels = 0;
        in >> kind >> n >> p >> levels;
        lgf_status st = LGF_OK;
        HostPlan H;
        if (kind == "single") {
            long long nb = 0;
            in >> nb;
            const std::vector<int32_t> b = read_blocks(in, nb);
            st = build_host(b.data(), nb, n, p, levels, H);
            if (st == LGF_OK) st = check_host(H);
        } else if (kind == "split") {
            long long ns = 0, ne = 0;
            in >> ns >> ne;
            const std::vector<int32_t> s = read_blocks(in, ns), e = read_blocks(in, ne);
            st = build_host(s.data(), ns, n, p, levels, H, e.data(), ne);
            if (st == LGF_OK) st = check_host(H);
        } else if (kind == "batch") {
            int count = 0;
            in >> count;
            std::vector<long long> nbs(count);
            for (auto& x : nbs) in >> x;
            std::vector<HostPlan> parts(count);
            for (int k = 0; k < count && st == LGF_OK; ++k) {
                const std::vector<int32_t> b = read_blocks(in, nbs[k]);
                st = build_host(b.data(), nbs[k], n, p, levels, parts[k]);
                if (st == LGF_OK) st = check_host(parts[k]);
            }
            if (st == LGF_OK) {
                H = concat(parts);
                st = check_host(H);
            }
        } else {
            std::fprintf(stderr, "unknown case kind %s\n", kind.c_str());
            return 2;
        }
        if (st != LGF_OK)
            std::printf("%d %s\n", (int)st, err_text().c_str());
        else
            print(H);
    }
    return 0;
}
