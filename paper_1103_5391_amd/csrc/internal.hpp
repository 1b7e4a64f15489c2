// Internal types shared by the host planner and the gfx950 kernels of libdmrgtst.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dmrg {

constexpr int kMaxKrylov = 64;      // largest kdim accepted
constexpr int kTile = 32;           // output tile edge of the block-product kernels
constexpr int kTile1N = 64;         // stage-1 tiles are kTile x kTile1N (one per wavefront),
constexpr int kTile1NN = 32;        // or kTile x kTile1NN (narrow: twice the tiles, each shorter)
constexpr int kTile2NN = 16;        // narrow stage-2 tiles are kTile x kTile2NN
constexpr int kChunk = 16;          // K depth of one FP64/FP32 chunk (4 MFMA K-steps of 4)
constexpr int kChunkMax = 32;       // K depth of one BF16 chunk (one 16x16x32 MFMA)
constexpr int kWaves = 4;           // waves per work group (split-K among them)
constexpr int kMultiRhs = 4;        // right-hand sides of the shared-operator stage kernels
constexpr int kVecThreads = 256;    // threads per block of the vector kernels
constexpr int kVecMaxBlocks = 1024; // blocks per problem of a vector pass (rows of partial sums)
constexpr int kDSlots = 15;         // basis slots per Lanczos reduction launch (4 values each,
                                    // plus 4: a row of 64, one per lane)
constexpr int kDVals = 4 * kDSlots + 4;   // values per partial row of a reduction launch
constexpr int kDMaxQ = (kMaxKrylov + kDSlots - 1) / kDSlots;   // reduction launches per iteration
#ifndef DMRG_RED_ELEMS
#define DMRG_RED_ELEMS 2
#endif
constexpr int kRedElems = DMRG_RED_ELEMS;  // complex elements per thread of a reduction pass
constexpr int kMaxTimes = 4;        // time points evaluated from one Krylov basis
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;   // device scratch per GPU of the
                                    // allocation-free entry point (the public header's
                                    // DMRG_NOALLOC_SCRATCH_BYTES)
constexpr int kXcd = 8;             // MI355X: 8 XCDs of 32 CUs, each with its own L2; work
                                    // group i of a launch runs on XCD i mod 8

// Element (r, c) of a matrix view inside a buffer.  Row-split views ("A" operands) place rows
// r >= split in a second plane at +poff; column-split views ("B" operands and outputs) place
// columns c >= split in a second plane at +poff.  split >= the extent means no second plane.
struct View {
    int64_t off;
    int64_t poff;
    int32_t ld;
    int32_t split;
};

// Operator factors are packed once per arithmetic in the order the MFMA lanes consume them:
// 16-row (or 16-column) panels, K chunks of depth CK (16 for FP64/FP32, 32 for BF16), and
// inside a chunk [g][r][t] with k = KPL g + t, KPL = CK / 4, so lane (g, r) reads its KPL
// values of one chunk as one contiguous piece (BF16: KPL hi values then KPL lo values).
// Rows (columns) are zero-padded to the tile and K to whole chunks, so operator loads never
// need bounds checks and padded products vanish.
constexpr int kPanel = 16;                        // rows (columns) per packed panel

// Stage 1 (right products) of one source block b:  T_b = X_b * R_b
//   X_b: 2d x e, rows 0..d-1 = real plane of Psi_b, rows d..2d-1 = imaginary plane
//   R_b: e x N, [H_E(q)^T | right factors of every term leaving b], packed (column panels)
//   T_b: workspace, column-major with both planes padded to dpad = d rounded up to a whole
//        K chunk (ld 2 dpad); the padding rows are zeroed once and never written, so the left
//        products read whole chunks of a column without bounds checks
struct S1Block {
    int32_t M, K, N, prob;
    int32_t nch, pad;   // K chunks of the packed factor
    View X;             // into the input vector
    int64_t Roff;       // into the packed right-factor buffer
    View T;             // into the workspace (row split like X)
};

// Stage 2 (left products and sum) of one output block b':
//   Y_b' (d' x 2e', columns e'.. = imaginary plane) = T0 + sum_seg Acat[:, seg] * B_seg
//   Acat: d' x Kcat, [H_S(p') | coef*sign*A of every term entering b'], packed (row panels,
//         every segment padded to whole chunks)
//   T0: the H_E columns of T_b'
struct S2Block {
    int32_t M, N, prob, nseg;
    int32_t seg0, nch;  // first segment, total K chunks of the packed factor
    int64_t Aoff;       // packed left-factor buffer
    View T0;            // into the workspace
    View Y;             // into the output vector
};

// One K segment of a stage-2 block: chunks ch0.. of Acat times the source view B (K x N).
struct Segment {
    int32_t K, ch0;
    int32_t src;        // 0: the input vector (diagonal H_S term), 1: the workspace
    int32_t pad;
    View B;
};

// One output tile of a register-tiled stage: rows m0.., columns n0.. of block blk; half: the
// tile has 16 rows instead of 32 (the last rows of a block, 16 or fewer).
struct Tile {
    int32_t blk, m0, n0, half;
};

// Work of the LDS-tiled block-product kernels: 64 x 64 output tiles, four wavefronts of 32 x 32
// sharing every K chunk of both operands through LDS.
constexpr int kLTile = 64;
constexpr int kLSlice = 16;         // most K chunks one stage-2 work group takes (16-deep chunks;
                                    // 8 of the 32-deep ones)

// Stage-1 tile: rows m0.., columns n0.. of block blk.
struct LItem1 {
    int32_t blk, m0, n0, pad;
};

// Stage-2 tile slice: K chunks [kc0, kc1) of the concatenated K of block blk for the output tile
// (m0, n0).  slot < 0: the slice is the whole K and the tile is written to y (plus T0); else
// the product is written to partial tile `slot` and summed by a reduction item.
struct LItem2 {
    int32_t blk, m0, n0, kc0, kc1, slot;
};

// Reduction of a split stage-2 tile: y = T0 + sum of partial tiles slot0 .. slot0 + nslice - 1
// (in that order).
struct LRed {
    int32_t blk, m0, n0, slot0, nslice, pad;
};

// Work of the LDS-staged (X) block-product family: work groups of four wavefronts whose
// operands are staged through double-buffered LDS in MFMA lane order.  Stage 1 takes the 64 x 64
// tiles of the LDS-tiled family (LItem1); stage 2 takes 64 x 32 output tiles, the long ones cut
// into two K slices that add into a zeroed output (two additions onto zero give the same bits in
// either order).
constexpr int kXTile2N = 32;        // stage-2 tile columns
constexpr int kXSplitChunks = 40;   // stage-2 tiles with more 16-deep K chunks run as two slices
constexpr int kXMaxItemChunks = 256;   // most chunks of one stage-2 item (its table in LDS); a
                                       // plan with longer items does not offer the family
// Source of one 16-deep K chunk of a stage-2 block: element (k, column n of plane p) of the
// chunk's segment at off + p poff + col ld + k, k counted from the block's first chunk (the
// segment's own start subtracted); src 0: the input vector (rows < K0 valid), 1: the workspace.
struct XChunk {
    int64_t off;
    int64_t poff;
    int32_t ld;
    int32_t src;
};
// One stage-2 work group: output tile (m0, n0) of block blk, K chunks [kc0, kc1); mode 0: the
// whole K, y = T0 + product; 1: first slice, y += T0 + product (atomic); 2: second slice,
// y += product (atomic).  ctab0: first entry of the block's chunk table.
struct XItem2 {
    int32_t blk, m0, n0, kc0, kc1, mode, ctab0, pad;
};
// A 64 x 32 output region of stage-2 block blk (at m0, n0) that split tiles add into: zeroed by
// extra work groups of the stage-1 launch.
struct XZero {
    int32_t blk, m0, n0, pad;
};

// Per-problem pointers for one launch of a stage (single problem: tables of length 1).
// Work of the K-split family (FP64): v_mfma_f64_4x4x4_4b_f64 with its four blocks taken as four
// slices of a 16-deep K chunk (partial sums added across the lanes once per tile), both operands
// of every stage packed in the instruction's lane order and streamed with 16-byte loads.
//   A operand (M x K): lane 16 k' + 4 b + x of the instruction for row group q holds
//     A(4 q + x, 16 c + 4 b + k'); B operand (K x N) likewise with column groups.
//   Piece (panel P of 32 rows or columns, chunk c): 512 doubles, [pair i][lane][2] with row
//     (column) group 2 i + s in element s of the pair; at off + (P pstride + c cstride) 512.
// Stage 1: T_b = X_b R_b as 32 x 32 tiles (or 16, 8, 4 rows / columns at block edges) of one
// wavefront; X_b comes from a pack of the input vector (written first by k_prepack), R_b from
// the packed right factors.  Its H_E columns go to T0 (d x 2e, column-major per block), the
// columns of every edge into that edge's packed stage-2 operand.  Stage 2: Y_b' = T0 + Acat Bcat,
// tiles of four wavefronts that deal the K chunks round-robin and add their partial tiles in
// LDS in a fixed order; the B piece of each chunk comes from a per-block chunk table (the
// block's own pack of the input vector for the H_S segment, then the edges' packs).
constexpr int kKPanel = 32;         // rows (columns) per packed panel: 8 groups of 4
constexpr int kKPiece = 512;        // doubles per (panel, chunk) piece
struct KPack {
    int64_t off;
    int32_t pstride, cstride;       // piece (P, c) at off + (P pstride + c cstride) kKPiece
};
// The family's index spaces start every piece of a block on a panel: stage 1's rows are the two
// planes of the block, each padded to dpad = d rounded up to 32 (plane p at rows p dpad..); its
// columns are the H_E columns, then every edge's, each padded to a multiple of 32; stage 2's
// columns are the two planes, each padded to epad = e rounded up to 32 (plane p at columns
// p epad..).  Padding rows and columns of the packs hold zeros and are never stored to, and no
// tile covers them (tiles cover groups of 4 up to the true extent): memory, not flops.
// Packing of the input vector for one psi block: xa = X_b (2 dpad x e) for stage 1, xb = the
// block as the H_S segment's B operand (d x 2 epad) for stage 2.
struct KXBlock {
    int32_t d, e, prob, dpad;
    int32_t epad, pad0;
    int64_t xoff;                   // block offset (complex elements) in the vector
    int64_t xplane;                 // offset of the vector's imaginary plane
    KPack xa, xb;                   // into the workspace
};
// One piece written by k_prepack: `which` 0: xa piece (P, c); 1: xb piece (P, c).
struct KPItem {
    int32_t blk, which, P, c;
};
// Stage-1 block: M = 2 dpad rows, K = e, N columns (segments padded to 32).
struct KS1Block {
    int32_t M, N, K, prob;
    int32_t d, e, nch, nedge;
    int32_t edge0, dpad, epad, pad0;
    KPack A;                        // the block's xa (workspace)
    KPack B;                        // packed right factors (operator buffer)
    int64_t t0off;                  // T0 (workspace): element (i, p epad + j) at + (p epad + j) d + i
};
// Stage-1 columns [col, col + e2) of a block (col a multiple of 32): one edge, whose stage-2
// operand (d_src x 2 e2pad, e2pad = e2 rounded up to 32) is packed at P (workspace,
// chunk-major: pstride 1, cstride = column panels of 2 e2pad).
struct KEdgeOut {
    int32_t col, e2, e2pad, pad0;
    KPack P;
};
// Stage-2 block: M = d' rows, N = 2 epad' columns, nch K chunks of the concatenated segments.
struct KS2Block {
    int32_t M, N, prob, nch;
    int32_t ctab0, e, epad, pad0;
    KPack A;                        // packed left factors (operator buffer)
    int64_t t0off;                  // T0 (workspace), as in KS1Block
    View Y;                         // into the output vector
};
// Tile of either stage: row groups g0 .. g0 + RQ - 1, column groups h0 .. h0 + CP - 1 (groups of
// 4), shape = 4 log2(RQ) + log2(CP) for RQ, CP in {1, 2, 4, 8} (RQ, CP >= 2: g0, h0 even).
// Stage 1 also names the tile's plane and column segment (-1: the H_E columns, else the edge
// index within the block's edges).
struct KTile {
    int32_t blk, g0, h0, shape;
    int32_t plane, seg, pad0, pad1;
};

struct ProbPtrs {
    const double* x;        // input vector
    double* y;              // output vector
    void* T;                // workspace (FP64 or FP32 elements)
    const void* Lops;       // packed left factors (stage 2), precision dependent type
    const void* Rops;       // packed right factors (stage 1)
    const int* skip;        // nonzero: skip all work of this problem (nullptr = never)
};

// One problem of a vector pass (fixed per handle; a batch concatenates them).  Blocks
// b0 .. b0 + nb - 1 of a launch work on this problem.
struct VecProb {
    double* V;            // basis slots: slot j at V + j * vstride
    double* w;            // matvec output / work vector
    double* part;         // block partial sums of this problem
    struct KState* st;
    int64_t n;            // complex length
    int64_t vstride;      // doubles between slots (2n)
    int32_t nb, b0;       // blocks of a streaming pass, first of them in the group's grid
    int32_t nbr, b0r;     // the same for the Lanczos reduction pass
};

// Launch description of the vector passes over a group of problems.
struct VecGroup {
    const VecProb* vp;    // device table [nprob]
    const int* bmap;      // device map block -> problem [nblk], nullptr for one problem
    const int* bmapr;     // the same for the reduction pass [nblkr]
    int nprob, nblk;      // problems, blocks of a pass (sum of nb)
    int nblkr;            // blocks of a reduction pass (sum of nbr)
    int combine_mult;     // blocks per pass block of the non-chained combination
    VecProb one;          // host copy of the descriptor when nprob == 1
};

// Reduced density matrix and truncation: one system sector (psi block) of the step.
struct DBlock {
    int32_t d, e;         // system states (rows of the psi block), environment states (columns)
    int64_t off;          // psi block offset in a vector (complex elements)
    int64_t aoff;         // its d x d complex matrices in the workspace (complex elements)
    int64_t eoff;         // its eigenvalues (sum of d over earlier sectors)
    int64_t toff;         // its back-transformation blocks T (complex elements)
};
// Back-transformation of a sector of d states: blocks of back_bt(d) reflectors (a block's
// reflectors fit in kBackVs complex elements), back_nblocks(d) of them.
constexpr int kBackVs = 2048;
__host__ __device__ constexpr int back_bt(int d) {
    return d <= kBackVs / 8 ? 8 : (d <= kBackVs / 4 ? 4 : 2);
}
__host__ __device__ constexpr int back_nblocks(int d) {
    return d >= 2 ? (d - 1 + back_bt(d) - 1) / back_bt(d) : 0;
}
// The back-transformation's work groups: kBackThreads threads, kBackLanes lanes per column of
// the eigenvector block, so back_cols(d) columns per work group (fewer when they would not fit
// the kBackLds complex elements of LDS).
constexpr int kBackThreads = 256;
constexpr int kBackLanes = 32;
constexpr int kBackCols = kBackThreads / kBackLanes;
constexpr int kBackLds = 4096;
__host__ __device__ constexpr int back_cols(int d) {
    return d * kBackCols <= kBackLds ? kBackCols : kBackLds / d;
}
struct DBackItem {        // one work group of the back-transformation: sector, first column
    int32_t blk, jb;
};
struct DTile {            // 16 x 16 tile of one sector's density matrix
    int32_t blk, i0, j0, pad;
};
constexpr int kDensMaxDim = 1024;   // largest system sector the eigen-decomposition accepts
constexpr int kDensMaxVec = 16;     // most target vectors of one density matrix
struct DensIn {            // target vectors (device, 2n doubles each) and their weights
    const double* v[kDensMaxVec];
    double w[kDensMaxVec];
};
constexpr int kDensRegMaxDim = 160;   // sectors up to this size take the register-resident kernel

// One 32 x 32 tile of a complex product C = alpha A B (+ C if acc) (FP64; complex operands
// have real parts at off and imaginary parts at off + im).  A modes: 0 complex column-major,
// A(i, k) at i + k lda; 1 conjugate transpose of a complex column-major X, A(i, k) =
// conj(X(k, i)) at k + i lda; 2 real column-major; 3 real transpose, A(i, k) = X(k, i) at
// k + i lda; 4 the identity (no memory).  B modes: 0 complex column-major, B(k, j) at
// k + j ldb; 1 transpose of a complex column-major X, B(k, j) = X(j, k) at j + k ldb; 2 real
// column-major; 3 real transpose.  C is complex column-major (ldc).  K = 0 gives a zero
// product.
enum ZMode { ZM_COL = 0, ZM_CT = 1, ZM_RCOL = 2, ZM_RT = 3, ZM_ID = 4 };
struct ZTile {
    int32_t M, N, K, m0, n0;
    int32_t amode, bmode, lda, ldb, ldc;
    int32_t acc, pad;
    double alpha;
    int64_t aoff, aim, boff, bim, coff, cim;
};
constexpr int kZTile = 32;
constexpr int kWftMaxVec = 16;      // vectors of one wave-function transformation call
struct ZPtrs {                      // per vector: the A, B and C buffers of one launch
    const double* a[kWftMaxVec];
    const double* b[kWftMaxVec];
    double* c[kWftMaxVec];
};

// One source block of a local term whose factors have at most one nonzero per row and per
// column (site operators on exact blocks and at the central sites): every element of the block
// goes to one element of the destination, scaled.  amap / bmap: offsets of the factors' maps
// (input index -> output index, -1 for none, with the value) in the system / environment
// tables, -1 for the identity.
struct SJob {
    int64_t src, dst;       // block offsets in x and y (complex elements)
    int32_t d, e, dout;     // source rows and columns, destination rows
    int32_t amap, bmap, pad;
    double alpha;
};

// Device state of one Krylov run on one problem.
struct KState {
    double alpha[kMaxKrylov];
    double beta[kMaxKrylov + 1];      // beta[0] = ||x||
    double scale[kMaxKrylov + 1];     // 1 / beta[j]: slot j of V holds beta[j] v_j
    double red[kDMaxQ * kDVals];      // totals of the reduction launches of one iteration
    double coef[kMaxTimes][2 * kMaxKrylov];  // c(t_x) = beta0 exp(-i T t_x) e_1
    double err_est;
    int32_t keff;
    int32_t broken;                   // 1 after breakdown (or zero input)
    int32_t kdim;
    int32_t exp_fail;                 // small exponential gave non-finite coefficients
    int32_t keff_min;                 // over all steps of one call
    int32_t any_break;                // over all steps of one call
    double beta0_first;               // ||x|| of the first step of one call
    double eig;                       // lowest eigenvalue of the Lanczos matrix (ground state)
    int32_t nonfinite;                // a step started from a vector with a non-finite norm
                                      // (any step of one call); the step is then run as a
                                      // zero vector
    int32_t pad;
};

}  // namespace dmrg
