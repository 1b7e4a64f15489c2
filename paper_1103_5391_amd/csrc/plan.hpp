// Host planner of libdmrgtst: sector tables, connection-term expansion, tile work lists and
// packed operator buffers for the two block-product stages of H_sb.psi.
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

// Block of an operator (or its transpose) leaving a sector: at(i, j) = element (i, j) of the
// (destination x source) block.
struct OpRef {
    int dst = -1;
    const double* data = nullptr;
    int ld = 0;          // leading dimension of the stored block
    bool transposed = false;
    double at(int i, int j) const {
        return transposed ? data[(int64_t)i * ld + j] : data[(int64_t)j * ld + i];
    }
};

// One connection term applied to one source block.
struct Edge {
    int src, dst, term;
    OpRef a, b;
    int col;             // first column of its right factor inside R_src (stage-1 output)
};

// Descriptors of the two stages for one K-chunk depth (16 for FP64 and FP32, 32 for the split
// bf16 arithmetics): the chunk structure decides the packed operator layout and sizes.  Offsets
// and sizes count one element per K index; an arithmetic that stores a value as `per` pieces
// scales them by per.
struct Packing {
    int ck = 0;
    std::vector<S1Block> s1;
    std::vector<S2Block> s2;
    std::vector<Segment> segs;
    int64_t A_elems = 0, R_elems = 0;          // packed operator values
    // LDS-tiled stage 2: slice length (chunks), tile slices, reductions of split tiles
    int slice = 0;
    std::vector<LItem2> l2;
    std::vector<LRed> lred;
    int nslots = 0;                            // partial tiles
    // LDS-staged family (16-deep chunks only): per-block chunk tables, stage-2 items, and the
    // output regions its split items add into
    std::vector<XChunk> xch;
    std::vector<XItem2> x2;
    std::vector<XZero> xz;
};

// Work of the K-split family (FP64): packs, descriptors and tiles.  Its packed factors follow the
// FP64 buffers of the other families (offsets count from the start of those buffers); its
// workspace layout (T0 per block, the edges' packed stage-2 operands, the packs of the input
// vector) starts at the workspace's first element.
struct KLists {
    std::vector<KXBlock> xblk;
    std::vector<KPItem> pitems;
    std::vector<KS1Block> s1;
    std::vector<KEdgeOut> eout;
    std::vector<KTile> t1;
    std::vector<KS2Block> s2;
    std::vector<int64_t> ctab;                 // per stage-2 chunk: workspace offset of its B
                                               // piece of column panel 0
    std::vector<KTile> t2;
    int64_t A_elems = 0, R_elems = 0;          // packed factor values after the FP64 packs
    int64_t T_size = 0;                        // workspace elements
};

struct Plan {
    HalfTable S, E;
    int target[2] = {0, 0};
    std::vector<TermSpec> terms;
    std::vector<PsiBlock> blocks;
    std::vector<int> block_of_S;               // S sector -> psi block or -1
    int64_t n = 0;                             // complex length
    std::vector<Edge> edges;
    std::vector<std::vector<int>> out_of, into;
    std::vector<int> N1;                       // stage-1 columns per source block
    std::vector<View> Tview;                   // stage-1 workspace view per block
    int64_t T_size = 0;                        // workspace elements (every family)
    int64_t T_base = 0;                        // of them, what the families other than the
                                               // K-split one use
    std::vector<Tile> tiles1, tiles1n, tiles2, tiles2n;   // register-tiled lists (wide, narrow)
    std::vector<LItem1> l1;                    // LDS-tiled stage-1 tiles (both packings)
    std::vector<double> w1, w2;                // per-block work estimates of the two stages
    Packing pk16, pk32;
    KLists kf;
    double flops = 0.0;                        // algorithmic flops per complex matvec: the
                                               // cheaper contraction order of every term
    double flops_exec = 0.0;                   // flops the two stages execute (right product
                                               // first for every term), padding excluded
    double flops1 = 0.0, flops2 = 0.0;         // of which stage 1 / stage 2
};

// Returns an empty string on success, else the reason the problem is invalid.
std::string build_plan(const dmrg_problem* pb, Plan& plan);

// Work lists of several plans merged into one launch per stage: problem i is plans[i] (its
// descriptors carry prob = i, its segments and blocks are renumbered), tiles in XCD order.
struct Merged {
    std::vector<S1Block> s1[2];               // per chunk depth (0: 16, 1: 32)
    std::vector<S2Block> s2[2];
    std::vector<Segment> segs[2];
    std::vector<Tile> tiles1, tiles1n, tiles2, tiles2n;
    std::vector<LItem1> l1;
    std::vector<LItem2> l2[2];
    std::vector<LRed> lred[2];
    int nslots[2] = {0, 0};
    std::vector<XChunk> xch;                  // LDS-staged family (16-deep chunks)
    std::vector<XItem2> x2;
    std::vector<XZero> xz;
    KLists kf;                                // K-split family
};
void merge_plans(const std::vector<const Plan*>& plans, Merged& out);

// Packed operator buffers for one arithmetic (raw bytes), kind = a dmrg_precision value: FP64
// and FP32 use the 16-deep packing, the split bf16 arithmetics (2 or 3 pieces per value) the
// 32-deep one.
void pack_operators(const Plan& plan, int kind, std::vector<uint8_t>& A, std::vector<uint8_t>& R);

}  // namespace dmrg
