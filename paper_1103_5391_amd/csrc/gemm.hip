// Grouped block products of H_sb.psi on gfx950 MFMA, in four arithmetics:
//   FP64    v_mfma_f64_16x16x4f64, FP64 workspace
//   FP32    v_mfma_f32_16x16x4f32, FP32 operands and workspace
//   BF16x3  v_mfma_f32_16x16x32_bf16 on split operands a = a0 + a1 (bf16 pieces, each the
//           rounding of what the previous leave): a0 b0 + a0 b1 + a1 b0 accumulated in FP32
//           (relative error about 2^-16), FP32 workspace
//   BF16x6  three pieces a = a0 + a1 + a2, the six products of total order <= 2
//           (about 2^-24, FP32-like), FP32 workspace
// The result of the second stage is always written in FP64.
//
// The Hamiltonian connections (Sec. IV) are applied as psi' = A psi B^T over (N_up, N_dn)
// symmetry blocks in two stages, each one launch over a list of output tiles:
//   stage 1  T_b  = X_b R_b        right products, X_b = [Re; Im] planes of the source block
//   stage 2  Y_b' = T0 + Acat Bcat left products summed over all terms entering the block
// Stage 1 gives each tile of 32 x 64 (or 32 x 32: twice the tiles, for better balance on small
// problems) to a work group of one wavefront (single-wave work groups let the dispatcher
// balance the compute units at the end of the launch).  In stage 2 a work group of four
// wavefronts owns one 32 x 32 tile (or 32 x 16, narrow) and deals its K chunks round-robin to the
// waves; the four partial tiles are summed in LDS in a fixed order (deterministic, no atomics).
//
// The operator factors are packed in MFMA lane order (mfma.hpp) and zero-padded so no operator
// load needs a bounds check.  The data operands are read in place: rows (stage 1) or columns
// (stage 2) are contiguous in K.  The stage-1 workspace is zero-padded to whole chunks; for the
// input vector out-of-range K indices are clamped to a valid element, whose product with the
// padded zeros vanishes.
#include "mfma.hpp"

namespace dmrg {

// ---------------------------------------------------------------------------------------
// stage 1: one 16 MI x 16 NJ tile (MI = 2, or 1 for a half-height tile; NJ = 4 wide, 2 narrow)
// per single-wavefront work group
// ---------------------------------------------------------------------------------------
template <class P, int MI, int NJ>
__device__ __forceinline__ void stage1_tile(const Tile& tl, const S1Block& B, const ProbPtrs& P_) {
    using op_t = typename P::op_t;
    using ws_t = typename P::ws_t;
    using acc_t = typename P::acc_t;
    using frag_t = typename P::frag_t;
    const int lane = threadIdx.x;
    const int g = lane >> 4, r = lane & 15;
    const double* __restrict__ X = P_.x;
    const int K = B.K;
    const int nch = (K + P::CK - 1) / P::CK;

    int64_t arow[MI];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
        const int m = min(tl.m0 + 16 * i + r, B.M - 1);
        const int pl = m >= B.X.split;
        arow[i] = B.X.off + pl * B.X.poff + (m - pl * B.X.split);
    }
    const op_t* pb = static_cast<const op_t*>(P_.Rops) + B.Roff * P::PER +
                     (((int64_t)(tl.n0 / kPanel) * nch) * 4 + g) * (kPanel * lane_elems<P>()) +
                     r * lane_elems<P>();
    const int64_t panel = (int64_t)nch * chunk_elems<P>();
    const int64_t ldx = B.X.ld;
    acc_t acc[MI][NJ];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) zero<P>(acc[mi][nj]);
    frag_t a[2][MI], b[2][NJ];
    auto load = [&](int c, frag_t (&fa)[MI], frag_t (&fb)[NJ]) {
        const int kb = c * P::CK + P::KPL * g;
#pragma unroll
        for (int i = 0; i < MI; ++i) {
            double v[P::KPL];
            load_clamped<P>(X, arow[i], kb, K, ldx, v);
            fa[i] = P::from(v);
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) fb[j] = P::load_op(pb + j * panel + (int64_t)c * chunk_elems<P>());
    };
    auto mma = [&](const frag_t (&fa)[MI], const frag_t (&fb)[NJ]) {
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj) acc[mi][nj] = P::mma(fa[mi], fb[nj], acc[mi][nj]);
    };
    // two register buffers, the next chunk always in flight (as in the stage-2 loop)
    load(0, a[0], b[0]);
    int c = 0;
    for (; c + 1 < nch; c += 2) {
        load(c + 1, a[1], b[1]);
        __builtin_amdgcn_sched_barrier(0);
        mma(a[0], b[0]);
        load(min(c + 2, nch - 1), a[0], b[0]);
        __builtin_amdgcn_sched_barrier(0);
        mma(a[1], b[1]);
    }
    if (c < nch) mma(a[0], b[0]);
    ws_t* __restrict__ T = static_cast<ws_t*>(P_.T);
    const View tv = B.T;
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) {
            const int n = tl.n0 + 16 * nj + r;
            if (n >= B.N) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = tl.m0 + 16 * mi + P::row(g, v);
                if (m < B.M) {
                    const int pl = m >= tv.split;
                    T[tv.off + pl * tv.poff + (int64_t)n * tv.ld + (m - pl * tv.split)] =
                        (ws_t)acc[mi][nj][v];
                }
            }
        }
}

template <class P, int NJ>
__global__ __launch_bounds__(64, 3) void stage1(const S1Block* __restrict__ blks,
                                                 const Tile* __restrict__ tiles, int ntiles,
                                                 const ProbPtrs* __restrict__ probs,
                                                 ProbPtrs single) {
    const int ti = blockIdx.x;
    if (ti >= ntiles) return;
    const Tile tl = tiles[ti];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const S1Block B = blks[tl.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    if (tl.half)
        stage1_tile<P, 1, NJ>(tl, B, P_);
    else
        stage1_tile<P, 2, NJ>(tl, B, P_);
}

// ---------------------------------------------------------------------------------------
// stage 2: one 32 x 32 (or 32 x 16) tile per work group, K chunks dealt round-robin to its waves
// ---------------------------------------------------------------------------------------
constexpr int kChunkTab = 256;   // workspace chunks of a block addressed through the LDS table
template <class P, int MI, int NJ, class Load>
__device__ __forceinline__ void kloop(typename P::acc_t (&acc)[MI][NJ], int c0, int step, int nch,
                                      Load load) {
    using frag_t = typename P::frag_t;
    if (c0 >= nch) return;
    const int last = c0 + (nch - 1 - c0) / step * step;
    frag_t a0[MI], b0[NJ], a1[MI], b1[NJ];
    auto mma = [&](const frag_t (&fa)[MI], const frag_t (&fb)[NJ]) {
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj) acc[mi][nj] = P::mma(fa[mi], fb[nj], acc[mi][nj]);
    };
    // Two register buffers, one exit test per pair of chunks: the chunk after the one being
    // multiplied is always in flight (the last prefetch is clamped and unused).  The
    // scheduling barriers keep each prefetch ahead of the products it overlaps; without them
    // the compiler moved the loads down to their products and waited for them there.
    load(c0, a0, b0);
    int c = c0;
    for (; c + step <= last; c += 2 * step) {
        load(c + step, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        mma(a0, b0);
        load(min(c + 2 * step, last), a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
    }
    if (c <= last) mma(a0, b0);   // odd count: chunk c is in a0
}

// One 16 MI x 16 NJ output tile (MI = 2, or 1 for a half-height tile) per work group of NW
// wavefronts (K chunks dealt round-robin); ctab and red live in the kernel's LDS.
template <class P, int MI, int NJ, int NW>
__device__ __forceinline__ void stage2_tile(const Tile& tl, const S2Block& B,
                                            const Segment* __restrict__ segs, const ProbPtrs& P_,
                                            int64_t (&ctab)[kChunkTab][3],
                                            double (&red)[NW][16 * NJ][kTile + 1]) {
    using op_t = typename P::op_t;
    using ws_t = typename P::ws_t;
    using acc_t = typename P::acc_t;
    using frag_t = typename P::frag_t;
    constexpr int TN = 16 * NJ;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int g = lane >> 4, r = lane & 15;
    const int split = B.Y.split;   // columns per plane of the output and of every source
    const ws_t* __restrict__ Tws = static_cast<const ws_t*>(P_.T);

    const op_t* pa[MI];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
        const int pnl = tl.m0 / kPanel + i;
        pa[i] = static_cast<const op_t*>(P_.Lops) + B.Aoff * P::PER +
                (((int64_t)pnl * B.nch) * 4 + g) * (kPanel * lane_elems<P>()) + r * lane_elems<P>();
    }
    int pl[NJ], col[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int n = min(tl.n0 + 16 * j + r, B.N - 1);
        pl[j] = n >= split;
        col[j] = n - pl[j] * split;
    }
    acc_t acc[MI][NJ];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) zero<P>(acc[mi][nj]);
    // pass 1: segment 0, the diagonal H_S term, reads the block itself from the input vector
    const Segment s0 = segs[B.seg0];
    const int nch0 = (s0.K + P::CK - 1) / P::CK;
    {
        int64_t bcol[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            bcol[j] = s0.B.off + pl[j] * s0.B.poff + (int64_t)col[j] * s0.B.ld;
        auto load = [&](int c, frag_t (&fa)[MI], frag_t (&fb)[NJ]) {
            const int64_t ga = (int64_t)c * chunk_elems<P>();
#pragma unroll
            for (int i = 0; i < MI; ++i) fa[i] = P::load_op(pa[i] + ga);
            const int kb = c * P::CK + P::KPL * g;
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                double v[P::KPL];
                load_clamped<P>(P_.x, bcol[j], kb, s0.K, 1, v);
                fb[j] = P::from(v);
            }
        };
        kloop<P, MI, NJ>(acc, wave, NW, nch0, load);
    }
    // pass 2: every workspace chunk of segments 1.. in one pipelined stream per wave (global
    // chunk c goes to wave c mod NW), its source view read from a per-chunk table in LDS (built
    // once per work group) instead of restarting the pipeline at every segment
    // ctab: per workspace chunk off - ch0 CK, poff, ld
    const int nT = B.nch - nch0;
    if (nT > 0 && nT <= kChunkTab) {
        for (int t = threadIdx.x; t < nT; t += blockDim.x) {
            const int c = nch0 + t;
            int si = 1;
            Segment sg = segs[B.seg0 + 1];
            while (c >= sg.ch0 + (sg.K + P::CK - 1) / P::CK) sg = segs[B.seg0 + ++si];
            ctab[t][0] = sg.B.off - (int64_t)sg.ch0 * P::CK;
            ctab[t][1] = sg.B.poff;
            ctab[t][2] = sg.B.ld;
        }
        __syncthreads();
        auto load = [&](int c, frag_t (&fa)[MI], frag_t (&fb)[NJ]) {
            const int64_t ga = (int64_t)c * chunk_elems<P>();
#pragma unroll
            for (int i = 0; i < MI; ++i) fa[i] = P::load_op(pa[i] + ga);
            const int64_t* e = ctab[c - nch0];
            const int64_t kb = (int64_t)c * P::CK + P::KPL * g;
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                double v[P::KPL];
                load_run<P>(Tws, e[0] + pl[j] * e[1] + (int64_t)col[j] * e[2] + kb, v);
                fb[j] = P::from(v);
            }
        };
        // first chunk >= nch0 owned by this wave
        const int cw = nch0 + ((wave - nch0) % NW + NW) % NW;
        kloop<P, MI, NJ>(acc, cw, NW, B.nch, load);
    } else {
        // very long K: one pipeline per segment
        for (int s = 1; s < B.nseg; ++s) {
            const Segment sg = segs[B.seg0 + s];
            int64_t bcol[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                bcol[j] = sg.B.off + pl[j] * sg.B.poff + (int64_t)col[j] * sg.B.ld;
            const int nch = (sg.K + P::CK - 1) / P::CK;
            const int c0 = ((wave - sg.ch0) % NW + NW) % NW;
            auto load = [&](int c, frag_t (&fa)[MI], frag_t (&fb)[NJ]) {
                const int64_t ga = (int64_t)(sg.ch0 + c) * chunk_elems<P>();
#pragma unroll
                for (int i = 0; i < MI; ++i) fa[i] = P::load_op(pa[i] + ga);
                const int kb = c * P::CK + P::KPL * g;
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    double v[P::KPL];
                    load_run<P>(Tws, bcol[j] + kb, v);
                    fb[j] = P::from(v);
                }
            };
            kloop<P, MI, NJ>(acc, c0, NW, nch, load);
        }
    }

#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                red[wave][16 * nj + r][16 * mi + P::row(g, v)] = (double)acc[mi][nj][v];
    __syncthreads();
    double* __restrict__ Y = P_.y;
    const View t0 = B.T0, yv = B.Y;
    const int m = threadIdx.x & 31;
    constexpr int kCols = 2 * NW;   // columns handled per pass of the work group
#pragma unroll
    for (int q = 0; q < TN / kCols; ++q) {
        const int n = (threadIdx.x >> 5) + kCols * q;
        const int gm = tl.m0 + m, gn = tl.n0 + n;
        if (gm < B.M && gn < B.N) {
            double v = red[0][n][m];
#pragma unroll
            for (int w = 1; w < NW; ++w) v += red[w][n][m];
            const int p = gn >= split;
            const int c = gn - p * split;
            const double init = (double)Tws[t0.off + p * t0.poff + (int64_t)c * t0.ld + gm];
            Y[yv.off + p * yv.poff + (int64_t)c * yv.ld + gm] = init + v;
        }
    }
}

template <class P, int NJ, int NW>
__global__ __launch_bounds__(64 * NW, 3) void stage2(const S2Block* __restrict__ blks,
                                                     const Segment* __restrict__ segs,
                                                     const Tile* __restrict__ tiles,
                                                     const ProbPtrs* __restrict__ probs,
                                                     ProbPtrs single) {
    const Tile tl = tiles[blockIdx.x];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const S2Block B = blks[tl.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    __shared__ int64_t ctab[kChunkTab][3];
    __shared__ double red[NW][16 * NJ][kTile + 1];
    if (tl.half)
        stage2_tile<P, 1, NJ, NW>(tl, B, segs, P_, ctab, red);
    else
        stage2_tile<P, 2, NJ, NW>(tl, B, segs, P_, ctab, red);
}

// ---------------------------------------------------------------------------------------
// stage 2 for several right-hand sides that share the operators (the chains of the 4-RHS
// mode): the tile list of the owners' plans, chain c of problem p at probs[NR p + c].  Each
// chunk's left-factor fragments are loaded once for all NR chains.  Every chain's products run
// in the order of the single-vector kernel above, so its results have the same bits.  A chain
// whose skip flag is set is computed (its buffers are allocated) but not stored.  (Stage 1
// stays per chain: four chains' accumulators and fragments there exceed the registers.)
// ---------------------------------------------------------------------------------------
// The problem pointers of chains c0 .. c0 + NR - 1 of a tile and which of them are live.
template <int NR>
__device__ __forceinline__ bool chain_ptrs(const ProbPtrs* __restrict__ probs, int prob, int c0,
                                           ProbPtrs (&PP)[NR], bool (&act)[NR]) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        PP[q] = probs[kMultiRhs * prob + c0 + q];
        act[q] = !(PP[q].skip && *PP[q].skip);
        any |= act[q];
    }
    return any;
}

// kloop for NR chains sharing the A fragments.
template <class P, int MI, int NJ, int NR, class Load>
__device__ __forceinline__ void kloop_mr(typename P::acc_t (&acc)[NR][MI][NJ], int c0, int step,
                                         int nch, Load load) {
    using frag_t = typename P::frag_t;
    if (c0 >= nch) return;
    const int last = c0 + (nch - 1 - c0) / step * step;
    frag_t a0[MI], b0[NR][NJ], a1[MI], b1[NR][NJ];
    auto mma = [&](const frag_t (&fa)[MI], const frag_t (&fb)[NR][NJ]) {
#pragma unroll
        for (int q = 0; q < NR; ++q)
#pragma unroll
            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                for (int nj = 0; nj < NJ; ++nj) acc[q][mi][nj] = P::mma(fa[mi], fb[q][nj], acc[q][mi][nj]);
    };
    load(c0, a0, b0);
    int c = c0;
    for (; c + step <= last; c += 2 * step) {
        load(c + step, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        mma(a0, b0);
        load(min(c + 2 * step, last), a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        mma(a1, b1);
    }
    if (c <= last) mma(a0, b0);
}

template <class P, int MI, int NJ, int NW, int NR>
__device__ __forceinline__ void stage2_tile_mr(const Tile& tl, const S2Block& B,
                                               const Segment* __restrict__ segs,
                                               const ProbPtrs (&PP)[NR], const bool (&act)[NR],
                                               int64_t (&ctab)[kChunkTab][3],
                                               double (&red)[NW][16 * NJ][kTile + 1]) {
    using op_t = typename P::op_t;
    using ws_t = typename P::ws_t;
    using acc_t = typename P::acc_t;
    using frag_t = typename P::frag_t;
    constexpr int TN = 16 * NJ;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int g = lane >> 4, r = lane & 15;
    const int split = B.Y.split;
    const op_t* pa[MI];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
        const int pnl = tl.m0 / kPanel + i;
        pa[i] = static_cast<const op_t*>(PP[0].Lops) + B.Aoff * P::PER +
                (((int64_t)pnl * B.nch) * 4 + g) * (kPanel * lane_elems<P>()) + r * lane_elems<P>();
    }
    int pl[NJ], col[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int n = min(tl.n0 + 16 * j + r, B.N - 1);
        pl[j] = n >= split;
        col[j] = n - pl[j] * split;
    }
    acc_t acc[NR][MI][NJ];
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj) zero<P>(acc[q][mi][nj]);
    // pass 1: segment 0 (H_S) from each chain's input vector
    const Segment s0 = segs[B.seg0];
    const int nch0 = (s0.K + P::CK - 1) / P::CK;
    {
        int64_t bcol[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j)
            bcol[j] = s0.B.off + pl[j] * s0.B.poff + (int64_t)col[j] * s0.B.ld;
        auto load = [&](int c, frag_t (&fa)[MI], frag_t (&fb)[NR][NJ]) {
            const int64_t ga = (int64_t)c * chunk_elems<P>();
#pragma unroll
            for (int i = 0; i < MI; ++i) fa[i] = P::load_op(pa[i] + ga);
            const int kb = c * P::CK + P::KPL * g;
#pragma unroll
            for (int q = 0; q < NR; ++q)
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    double v[P::KPL];
                    load_clamped<P>(PP[q].x, bcol[j], kb, s0.K, 1, v);
                    fb[q][j] = P::from(v);
                }
        };
        kloop_mr<P, MI, NJ, NR>(acc, wave, NW, nch0, load);
    }
    // pass 2: the workspace chunks of segments 1.. from each chain's stage-1 intermediate
    const int nT = B.nch - nch0;
    if (nT > 0 && nT <= kChunkTab) {
        for (int t = threadIdx.x; t < nT; t += blockDim.x) {
            const int c = nch0 + t;
            int si = 1;
            Segment sg = segs[B.seg0 + 1];
            while (c >= sg.ch0 + (sg.K + P::CK - 1) / P::CK) sg = segs[B.seg0 + ++si];
            ctab[t][0] = sg.B.off - (int64_t)sg.ch0 * P::CK;
            ctab[t][1] = sg.B.poff;
            ctab[t][2] = sg.B.ld;
        }
        __syncthreads();
        auto load = [&](int c, frag_t (&fa)[MI], frag_t (&fb)[NR][NJ]) {
            const int64_t ga = (int64_t)c * chunk_elems<P>();
#pragma unroll
            for (int i = 0; i < MI; ++i) fa[i] = P::load_op(pa[i] + ga);
            const int64_t* e = ctab[c - nch0];
            const int64_t kb = (int64_t)c * P::CK + P::KPL * g;
#pragma unroll
            for (int q = 0; q < NR; ++q)
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    double v[P::KPL];
                    load_run<P>(static_cast<const ws_t*>(PP[q].T),
                                e[0] + pl[j] * e[1] + (int64_t)col[j] * e[2] + kb, v);
                    fb[q][j] = P::from(v);
                }
        };
        const int cw = nch0 + ((wave - nch0) % NW + NW) % NW;
        kloop_mr<P, MI, NJ, NR>(acc, cw, NW, B.nch, load);
    } else {
        for (int s = 1; s < B.nseg; ++s) {
            const Segment sg = segs[B.seg0 + s];
            int64_t bcol[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                bcol[j] = sg.B.off + pl[j] * sg.B.poff + (int64_t)col[j] * sg.B.ld;
            const int nch = (sg.K + P::CK - 1) / P::CK;
            const int c0 = ((wave - sg.ch0) % NW + NW) % NW;
            auto load = [&](int c, frag_t (&fa)[MI], frag_t (&fb)[NR][NJ]) {
                const int64_t ga = (int64_t)(sg.ch0 + c) * chunk_elems<P>();
#pragma unroll
                for (int i = 0; i < MI; ++i) fa[i] = P::load_op(pa[i] + ga);
                const int kb = c * P::CK + P::KPL * g;
#pragma unroll
                for (int q = 0; q < NR; ++q)
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        double v[P::KPL];
                        load_run<P>(static_cast<const ws_t*>(PP[q].T), bcol[j] + kb, v);
                        fb[q][j] = P::from(v);
                    }
            };
            kloop_mr<P, MI, NJ, NR>(acc, c0, NW, nch, load);
        }
    }
    // the waves' partial tiles summed in LDS in a fixed order, one chain after another
    const View t0 = B.T0, yv = B.Y;
    const int m = threadIdx.x & 31;
    constexpr int kCols = 2 * NW;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (!act[q]) continue;                          // the same in every thread
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    red[wave][16 * nj + r][16 * mi + P::row(g, v)] = (double)acc[q][mi][nj][v];
        __syncthreads();
        const ws_t* __restrict__ Tws = static_cast<const ws_t*>(PP[q].T);
        double* __restrict__ Y = PP[q].y;
#pragma unroll
        for (int qq = 0; qq < TN / kCols; ++qq) {
            const int n = (threadIdx.x >> 5) + kCols * qq;
            const int gm = tl.m0 + m, gn = tl.n0 + n;
            if (gm < B.M && gn < B.N) {
                double v = red[0][n][m];
#pragma unroll
                for (int w = 1; w < NW; ++w) v += red[w][n][m];
                const int p = gn >= split;
                const int c = gn - p * split;
                const double init = (double)Tws[t0.off + p * t0.poff + (int64_t)c * t0.ld + gm];
                Y[yv.off + p * yv.poff + (int64_t)c * yv.ld + gm] = init + v;
            }
        }
        __syncthreads();                                // red is written again for the next chain
    }
}

template <class P, int NJ, int NW, int NR>
__global__ __launch_bounds__(64 * NW, 2) void stage2_mr(const S2Block* __restrict__ blks,
                                                        const Segment* __restrict__ segs,
                                                        const Tile* __restrict__ tiles,
                                                        const ProbPtrs* __restrict__ probs) {
    const Tile tl = tiles[blockIdx.x];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const S2Block B = blks[tl.blk];
    ProbPtrs PP[NR];
    bool act[NR];
    if (!chain_ptrs<NR>(probs, B.prob, NR * (int)blockIdx.y, PP, act)) return;
    __shared__ int64_t ctab[kChunkTab][3];
    __shared__ double red[NW][16 * NJ][kTile + 1];
    if (tl.half)
        stage2_tile_mr<P, 1, NJ, NW, NR>(tl, B, segs, PP, act, ctab, red);
    else
        stage2_tile_mr<P, 2, NJ, NW, NR>(tl, B, segs, PP, act, ctab, red);
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
namespace {

template <class P>
hipError_t launch1(int narrow, const S1Block* blks, const Tile* tiles, int ntiles,
                   const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    if (narrow)
        hipLaunchKernelGGL((stage1<P, kTile1NN / 16>), dim3(ntiles), dim3(64), 0, st, blks, tiles,
                           ntiles, probs, single);
    else
        hipLaunchKernelGGL((stage1<P, kTile1N / 16>), dim3(ntiles), dim3(64), 0, st, blks, tiles,
                           ntiles, probs, single);
    return hipGetLastError();
}

template <class P>
hipError_t launch2(int narrow, const S2Block* blks, const Segment* segs, const Tile* tiles,
                   int ntiles, const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    if (narrow)
        hipLaunchKernelGGL((stage2<P, kTile2NN / 16, kWaves>), dim3(ntiles), dim3(64 * kWaves), 0,
                           st, blks, segs, tiles, probs, single);
    else
        hipLaunchKernelGGL((stage2<P, kTile / 16, kWaves>), dim3(ntiles), dim3(64 * kWaves), 0, st,
                           blks, segs, tiles, probs, single);
    return hipGetLastError();
}

}  // namespace

// Stage 2 of the chains of the 4-RHS mode in one launch (FP64, narrow tiles): the owners' tile
// list, chain c of problem p at probs[kMultiRhs p + c].
hipError_t launch_stage2_mr(const S2Block* blks, const Segment* segs, const Tile* tiles,
                            int ntiles, const ProbPtrs* probs, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    // all chains in one work group (two per work group, with a second grid row for the other
    // two, measured the same)
    constexpr int NR = kMultiRhs;
    hipLaunchKernelGGL((stage2_mr<PF64, kTile2NN / 16, kWaves, NR>), dim3(ntiles, kMultiRhs / NR),
                       dim3(64 * kWaves), 0, st, blks, segs, tiles, probs);
    return hipGetLastError();
}

// prec: 0 FP64, 1 FP32, 2 BF16x3, 3 BF16x6 (the operator buffers and workspace must match);
// narrow: the tiles are kTile x kTile1NN (else kTile x kTile1N)
hipError_t launch_stage1(int prec, int narrow, const S1Block* blks, const Tile* tiles, int ntiles,
                         const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    switch (prec) {
        case 0: return launch1<PF64>(narrow, blks, tiles, ntiles, probs, single, st);
        case 1: return launch1<PF32>(narrow, blks, tiles, ntiles, probs, single, st);
        case 2: return launch1<PBF3>(narrow, blks, tiles, ntiles, probs, single, st);
        default: return launch1<PBF6>(narrow, blks, tiles, ntiles, probs, single, st);
    }
}

// narrow: the tiles are kTile x kTile2NN (else kTile x kTile)
hipError_t launch_stage2(int prec, int narrow, const S2Block* blks, const Segment* segs,
                         const Tile* tiles, int ntiles, const ProbPtrs* probs, ProbPtrs single,
                         hipStream_t st) {
    switch (prec) {
        case 0: return launch2<PF64>(narrow, blks, segs, tiles, ntiles, probs, single, st);
        case 1: return launch2<PF32>(narrow, blks, segs, tiles, ntiles, probs, single, st);
        case 2: return launch2<PBF3>(narrow, blks, segs, tiles, ntiles, probs, single, st);
        default: return launch2<PBF6>(narrow, blks, segs, tiles, ntiles, probs, single, st);
    }
}

}  // namespace dmrg
