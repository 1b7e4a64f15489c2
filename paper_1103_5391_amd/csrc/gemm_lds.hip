// LDS-tiled block products of H_sb.psi on gfx950: the two stages of gemm.hip on 64 x 64
// output tiles.
//
// A work group of four wavefronts (2 x 2, each 32 x 32 of the tile) loads every K chunk of both
// operands once into LDS, already in MFMA fragment order, and all four waves multiply from
// there.  Per MFMA this moves half the operand bytes from L2 of a private 32 x 32 tile per work
// group.  Chunks move in groups of D: the D chunks of the next group are requested into
// registers, the D chunks of the current group are multiplied from LDS (D x 16 MFMAs per wave to
// cover the load latency), then the registers are written over the consumed LDS buffers
// between two barriers.  Row and column panels (16) of the tile that lie beyond the block are
// neither loaded nor multiplied, so padding costs at most 15 rows and columns per block edge.
//
// Stage 2 (K = concatenated left factors, up to ~1300 at m = 1000) splits long K ranges into
// slices run by separate work groups: each slice writes a partial tile, and a reduction launch
// adds T0 and the partial tiles of a tile in slice order (deterministic, no atomics).  Tiles
// with a single slice write y directly.
#include "mfma.hpp"

namespace dmrg {

namespace {

// Chunks per prefetch group: the LDS holds one group (D buffers of both operands).
template <class P>
constexpr int group_depth() {
    return sizeof(typename P::frag_t) > 32 ? 2 : (sizeof(typename P::frag_t) > 16 ? 3 : 4);
}

template <class P>
struct LdsTiles {
    typename P::frag_t A[group_depth<P>()][4][64];   // [buffer][row panel][lane]
    typename P::frag_t B[group_depth<P>()][4][64];   // [buffer][column panel][lane]
};

// One K chunk of the wave's 32 x 32 sub-tile from LDS buffer `buf`; vm, vn: valid 16-row and
// 16-column panels of the sub-tile (wave-uniform).
template <class P>
__device__ __forceinline__ void mma_chunk(typename P::acc_t (&acc)[2][2], const LdsTiles<P>& sm,
                                          int buf, int wm, int wn, int lane, int vm, int vn) {
    using frag_t = typename P::frag_t;
    frag_t fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        fa[i] = sm.A[buf][2 * wm + i][lane];
        fb[i] = sm.B[buf][2 * wn + i][lane];
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
            if (mi < vm && nj < vn) acc[mi][nj] = P::mma(fa[mi], fb[nj], acc[mi][nj]);
}

// Runs chunks [c0, c1) through the grouped LDS pipeline.  load(c, d) requests chunk c into
// register set d, store(d) writes register set d into LDS buffer d.
template <class P, class Load, class Store>
__device__ __forceinline__ void lds_pipeline(typename P::acc_t (&acc)[2][2], LdsTiles<P>& sm,
                                             int c0, int c1, int wm, int wn, int lane, int vm,
                                             int vn, Load load, Store store) {
    constexpr int D = group_depth<P>();
#pragma unroll
    for (int d = 0; d < D; ++d) load(min(c0 + d, c1 - 1), d);
#pragma unroll
    for (int d = 0; d < D; ++d) store(d);
    __syncthreads();
    for (int c = c0; c < c1; c += D) {
        // next group in flight (indices clamped: the last group may repeat its final chunk)
#pragma unroll
        for (int d = 0; d < D; ++d) load(min(c + D + d, c1 - 1), d);
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (c + d < c1) mma_chunk<P>(acc, sm, d, wm, wn, lane, vm, vn);
        __syncthreads();   // every wave is done with the group's buffers
        if (c + D < c1) {
#pragma unroll
            for (int d = 0; d < D; ++d) store(d);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int clamp2(int v) { return v < 0 ? 0 : (v > 2 ? 2 : v); }

}  // namespace

// ---------------------------------------------------------------------------------------
// stage 1: T_b = X_b R_b on 64 x 64 tiles (K = e <= a few hundred: no split)
// ---------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(256, 3) void stage1_lds(const S1Block* __restrict__ blks,
                                                     const LItem1* __restrict__ items,
                                                     const ProbPtrs* __restrict__ probs,
                                                     ProbPtrs single) {
    using op_t = typename P::op_t;
    using ws_t = typename P::ws_t;
    using acc_t = typename P::acc_t;
    using frag_t = typename P::frag_t;
    const LItem1 it = items[blockIdx.x];
    if (it.blk < 0) return;   // padding of the XCD-ordered list
    const S1Block B = blks[it.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    __shared__ LdsTiles<P> sm;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int g = lane >> 4, r = lane & 15;
    const int mval = min(4, (B.M - it.m0 + 15) / 16), nval = min(4, (B.N - it.n0 + 15) / 16);
    const int vm = clamp2(mval - 2 * wm), vn = clamp2(nval - 2 * wn);
    const int K = B.K, nch = (K + P::CK - 1) / P::CK;

    // loader roles: wave w brings row panel w of X (lane (g, r): row 16 w + r, KPL values of
    // its K quarter) and column panel w of R (the lane's packed piece)
    const bool a_on = wave < mval, b_on = wave < nval;
    const int arow_m = min(it.m0 + 16 * wave + r, B.M - 1);
    const int apl = arow_m >= B.X.split;
    const int64_t arow = B.X.off + apl * B.X.poff + (arow_m - apl * B.X.split);
    const int64_t ldx = B.X.ld;
    const double* __restrict__ X = P_.x;
    const op_t* __restrict__ pb = static_cast<const op_t*>(P_.Rops) + B.Roff * P::PER +
                                  (((int64_t)(it.n0 / kPanel + wave) * nch) * 4 + g) *
                                      (kPanel * lane_elems<P>()) +
                                  r * lane_elems<P>();
    // loads only request data (raw values in registers); conversion to the MFMA input type
    // happens when the group is written to LDS, after the products of the previous group
    constexpr int D = group_depth<P>();
    double xa[D][P::KPL];
    frag_t rb[D];
    auto load = [&](int c, int d) {
        if (a_on) load_clamped<P>(X, arow, c * P::CK + P::KPL * g, K, ldx, xa[d]);
        if (b_on) rb[d] = P::load_op(pb + (int64_t)c * chunk_elems<P>());
    };
    auto store = [&](int d) {
        if (a_on) sm.A[d][wave][lane] = P::from(xa[d]);
        if (b_on) sm.B[d][wave][lane] = rb[d];
    };

    acc_t acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) zero<P>(acc[mi][nj]);
    lds_pipeline<P>(acc, sm, 0, nch, wm, wn, lane, vm, vn, load, store);

    ws_t* __restrict__ T = static_cast<ws_t*>(P_.T);
    const View tv = B.T;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            const int n = it.n0 + 32 * wn + 16 * nj + r;
            if (n >= B.N) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = it.m0 + 32 * wm + 16 * mi + P::row(g, v);
                if (m < B.M) {
                    const int pl = m >= tv.split;
                    T[tv.off + pl * tv.poff + (int64_t)n * tv.ld + (m - pl * tv.split)] =
                        (ws_t)acc[mi][nj][v];
                }
            }
        }
}

// ---------------------------------------------------------------------------------------
// stage 2: Y_b' = T0 + Acat Bcat on 64 x 64 tiles, K chunks [kc0, kc1) per work group
// ---------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(256, 3) void stage2_lds(const S2Block* __restrict__ blks,
                                                     const Segment* __restrict__ segs,
                                                     const LItem2* __restrict__ items,
                                                     const ProbPtrs* __restrict__ probs,
                                                     ProbPtrs single, double* __restrict__ part) {
    using op_t = typename P::op_t;
    using ws_t = typename P::ws_t;
    using acc_t = typename P::acc_t;
    using frag_t = typename P::frag_t;
    const LItem2 it = items[blockIdx.x];
    if (it.blk < 0) return;   // padding of the XCD-ordered list
    const S2Block B = blks[it.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    __shared__ LdsTiles<P> sm;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int g = lane >> 4, r = lane & 15;
    const int split = B.Y.split;   // columns per plane of the output and of every source
    const ws_t* __restrict__ Tws = static_cast<const ws_t*>(P_.T);
    const int mval = min(4, (B.M - it.m0 + 15) / 16), nval = min(4, (B.N - it.n0 + 15) / 16);
    const int vm = clamp2(mval - 2 * wm), vn = clamp2(nval - 2 * wn);

    // loader roles: wave w brings row panel w of Acat (the lane's packed piece); thread t brings
    // column t / 4 of the tile, K quarter t % 4 (KPL values), as the fragment of lane
    // (t % 4, t / 4 % 16) of column panel t / 64
    const bool a_on = wave < mval;
    const op_t* __restrict__ pa = static_cast<const op_t*>(P_.Lops) + B.Aoff * P::PER +
                                  (((int64_t)(it.m0 / kPanel + wave) * B.nch) * 4 + g) *
                                      (kPanel * lane_elems<P>()) +
                                  r * lane_elems<P>();
    const int bn = tid >> 2, bq = tid & 3;
    const int ncol = min(it.n0 + bn, B.N - 1);
    const int bpl = ncol >= split;
    const int bcol = ncol - bpl * split;
    const int bp = bn >> 4, bl = bq * 16 + (bn & 15);

    // pass 1: chunks of segment 0 (the diagonal H_S term, read from the input vector, clamped
    // to the block and scaled like the workspace); pass 2: the workspace chunks, addressed
    // through a per-chunk table of source views (a slice has at most kLSlice chunks)
    const Segment s0 = segs[B.seg0];
    const int x_end = min(it.kc1, (s0.K + P::CK - 1) / P::CK);
    const int t_beg = max(it.kc0, x_end);
    __shared__ int64_t ctab[kLSlice][3];   // per workspace chunk: off - ch0 CK, poff, ld
    if (tid < it.kc1 - t_beg) {
        const int c = t_beg + tid;
        int si = 1;
        Segment sg = segs[B.seg0 + 1];
        while (c >= sg.ch0 + (sg.K + P::CK - 1) / P::CK) sg = segs[B.seg0 + ++si];
        ctab[tid][0] = sg.B.off - (int64_t)sg.ch0 * P::CK;
        ctab[tid][1] = sg.B.poff;
        ctab[tid][2] = sg.B.ld;
    }
    __syncthreads();

    constexpr int D = group_depth<P>();
    frag_t ra[D];
    double xb[D][P::KPL];
    ws_t tb[D][P::KPL];
    auto load_a = [&](int c, int d) {
        if (a_on) ra[d] = P::load_op(pa + (int64_t)c * chunk_elems<P>());
    };
    const int64_t xbase = s0.B.off + bpl * s0.B.poff + (int64_t)bcol * s0.B.ld;
    auto load_x = [&](int c, int d) {
        load_a(c, d);
        load_clamped<P>(P_.x, xbase, c * P::CK + P::KPL * bq, s0.K, 1, xb[d]);
    };
    auto store_x = [&](int d) {
        if (a_on) sm.A[d][wave][lane] = ra[d];
        sm.B[d][bp][bl] = P::from(xb[d]);
    };
    auto load_t = [&](int c, int d) {
        load_a(c, d);
        const int64_t* e = ctab[c - t_beg];
        const int64_t base = e[0] + bpl * e[1] + (int64_t)bcol * e[2] + c * P::CK + P::KPL * bq;
#pragma unroll
        for (int t = 0; t < P::KPL; ++t) tb[d][t] = ldg(Tws, base + t);
    };
    auto store_t = [&](int d) {
        if (a_on) sm.A[d][wave][lane] = ra[d];
        double v[P::KPL];
#pragma unroll
        for (int t = 0; t < P::KPL; ++t) v[t] = (double)tb[d][t];
        sm.B[d][bp][bl] = P::from(v);
    };

    acc_t acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) zero<P>(acc[mi][nj]);
    if (it.kc0 < x_end) lds_pipeline<P>(acc, sm, it.kc0, x_end, wm, wn, lane, vm, vn, load_x, store_x);
    if (t_beg < it.kc1) lds_pipeline<P>(acc, sm, t_beg, it.kc1, wm, wn, lane, vm, vn, load_t, store_t);

    if (it.slot < 0) {
        double* __restrict__ Y = P_.y;
        const View t0 = B.T0, yv = B.Y;
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < 2; ++nj) {
                const int n = it.n0 + 32 * wn + 16 * nj + r;
                if (n >= B.N) continue;
                const int p = n >= split;
                const int cc = n - p * split;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = it.m0 + 32 * wm + 16 * mi + P::row(g, v);
                    if (m < B.M) {
                        const double init = (double)Tws[t0.off + p * t0.poff + (int64_t)cc * t0.ld + m];
                        Y[yv.off + p * yv.poff + (int64_t)cc * yv.ld + m] = init + (double)acc[mi][nj][v];
                    }
                }
            }
    } else {
        // partial tile, column-major 64 x 64
        double* __restrict__ pt = part + (int64_t)it.slot * (kLTile * kLTile);
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < 2; ++nj) {
                const int n = 32 * wn + 16 * nj + r;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int m = 32 * wm + 16 * mi + P::row(g, v);
                    pt[n * kLTile + m] = (double)acc[mi][nj][v];
                }
            }
    }
}

// y = T0 + partial tiles in slice order, for the split tiles of stage 2.
template <typename ws_t>
__global__ __launch_bounds__(256) void stage2_reduce(const S2Block* __restrict__ blks,
                                                     const LRed* __restrict__ reds,
                                                     const ProbPtrs* __restrict__ probs,
                                                     ProbPtrs single,
                                                     const double* __restrict__ part) {
    const LRed rd = reds[blockIdx.x];
    const S2Block B = blks[rd.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    const ws_t* __restrict__ Tws = static_cast<const ws_t*>(P_.T);
    double* __restrict__ Y = P_.y;
    const View t0 = B.T0, yv = B.Y;
    const int split = yv.split;
#pragma unroll 4
    for (int q = 0; q < kLTile * kLTile / 256; ++q) {
        const int e = (int)threadIdx.x + 256 * q;
        const int row = e & (kLTile - 1), col = e / kLTile;
        const int m = rd.m0 + row, n = rd.n0 + col;
        if (m < B.M && n < B.N) {
            const int p = n >= split;
            const int cc = n - p * split;
            double s = (double)Tws[t0.off + p * t0.poff + (int64_t)cc * t0.ld + m];
            for (int sl = 0; sl < rd.nslice; ++sl)
                s += part[(int64_t)(rd.slot0 + sl) * (kLTile * kLTile) + e];
            Y[yv.off + p * yv.poff + (int64_t)cc * yv.ld + m] = s;
        }
    }
}

// ---------------------------------------------------------------------------------------
// launchers (prec: 0 FP64, 1 FP32, 2 BF16x3, 3 BF16x6)
// ---------------------------------------------------------------------------------------
namespace {

template <class P>
hipError_t launch1l(const S1Block* blks, const LItem1* items, int nitems, const ProbPtrs* probs,
                    ProbPtrs single, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(stage1_lds<P>, dim3(nitems), dim3(256), 0, st, blks, items, probs, single);
    return hipGetLastError();
}

template <class P>
hipError_t launch2l(const S2Block* blks, const Segment* segs, const LItem2* items, int nitems,
                    const LRed* reds, int nred, const ProbPtrs* probs, ProbPtrs single,
                    double* part, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(stage2_lds<P>, dim3(nitems), dim3(256), 0, st, blks, segs, items, probs,
                       single, part);
    if (nred > 0)
        hipLaunchKernelGGL(stage2_reduce<typename P::ws_t>, dim3(nred), dim3(256), 0, st, blks,
                           reds, probs, single, (const double*)part);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stage1_lds(int prec, const S1Block* blks, const LItem1* items, int nitems,
                             const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    switch (prec) {
        case 0: return launch1l<PF64>(blks, items, nitems, probs, single, st);
        case 1: return launch1l<PF32>(blks, items, nitems, probs, single, st);
        case 2: return launch1l<PBF3>(blks, items, nitems, probs, single, st);
        default: return launch1l<PBF6>(blks, items, nitems, probs, single, st);
    }
}

hipError_t launch_stage2_lds(int prec, const S2Block* blks, const Segment* segs,
                             const LItem2* items, int nitems, const LRed* reds, int nred,
                             const ProbPtrs* probs, ProbPtrs single, double* part,
                             hipStream_t st) {
    switch (prec) {
        case 0: return launch2l<PF64>(blks, segs, items, nitems, reds, nred, probs, single, part, st);
        case 1: return launch2l<PF32>(blks, segs, items, nitems, reds, nred, probs, single, part, st);
        case 2: return launch2l<PBF3>(blks, segs, items, nitems, reds, nred, probs, single, part, st);
        default: return launch2l<PBF6>(blks, segs, items, nitems, reds, nred, probs, single, part, st);
    }
}

}  // namespace dmrg
