// Host planner of libdmrgtst: sector tables, connection-term expansion, packed operator
// buffers and tile work lists for the two block-product stages of H_sb.psi.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dmrgtst.h"
#include "internal.hpp"

namespace dmrg {

struct HalfTable {
    int nsec = 0;
    std::vector<int> nup, ndn, dim;
    std::vector<int64_t> hoff;                 // offset of each H block in H
    std::vector<double> H;
    std::map<std::pair<int, int>, int> index;  // (N_up, N_dn) -> sector
    struct Op {
        int dq[2];
        std::vector<int64_t> boff;             // per source sector, -1 if no image
        std::vector<double> data;
    };
    std::vector<Op> ops;

    int find(int a, int b) const {
        auto it = index.find({a, b});
        return it == index.end() ? -1 : it->second;
    }
    int parity(int p) const { return ((nup[p] + ndn[p]) & 1) ? -1 : 1; }
};

struct TermSpec {
    double coef;
    int opS, transS, opE, transE, fermionic;
};

struct PsiBlock {
    int p, q, d, e;
    int64_t off;
};

// Everything the device needs for H_sb.psi in one precision-independent form (FP64 data).
struct Plan {
    HalfTable S, E;
    int target[2] = {0, 0};
    std::vector<TermSpec> terms;
    std::vector<PsiBlock> blocks;
    std::vector<int> block_of_S;               // S sector -> psi block or -1
    int64_t n = 0;                             // complex length
    // stage 1
    std::vector<S1Block> s1;
    std::vector<double> R;                     // packed right factors
    std::vector<Tile> tiles1;
    // stage 2
    std::vector<S2Block> s2;
    std::vector<Segment> segs;
    std::vector<double> A;                     // packed left factors
    std::vector<Tile> tiles2;
    int64_t T_size = 0;                        // workspace doubles
    double flops = 0.0;                        // algorithmic flops per complex matvec
    double flops1 = 0.0, flops2 = 0.0;         // of which stage 1 / stage 2
};

// Returns an empty string on success, else the reason the problem is invalid.
std::string build_plan(const dmrg_problem* pb, Plan& plan);

}  // namespace dmrg
