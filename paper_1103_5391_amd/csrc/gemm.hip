// Grouped block products of H_sb.psi on gfx950 FP64 MFMA (v_mfma_f64_16x16x4f64).
//
// The Hamiltonian connections (Sec. IV) are applied as psi' = A psi B^T over (N_up, N_dn)
// symmetry blocks in two stages, each one launch over a list of 32 x 32 output tiles:
//   stage 1  T_b  = X_b R_b        right products, X_b = [Re; Im] planes of the source block
//   stage 2  Y_b' = T0 + Acat Bcat left products summed over all terms entering the block
// Stage 1 gives each wavefront its own 32 x 64 tile.  In stage 2 a work group of four wavefronts owns
// one tile and deals its K chunks round-robin to the waves; the four partial tiles are summed
// in LDS in a fixed order (deterministic, no atomics).  Each wave holds 2 x 2 MFMA
// accumulators (32 x 32).
//
// Inside one 4-deep MFMA step the K index each lane group supplies is free as long as A and B
// agree, so lane group g takes k = 4g + t at step t.  The operator factors are packed in
// exactly that order (see internal.hpp), so lane (g, r) reads the four K values of a chunk as
// 32 contiguous bytes, and they are zero-padded so no operator load needs a bounds check.
// The data operands (the vector and the stage-1 workspace) are read in place: rows (stage 1)
// or columns (stage 2) are contiguous in K, and out-of-range indices are clamped to a valid
// element, whose product with the padded zeros vanishes.
#include "internal.hpp"

namespace dmrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef const double __attribute__((address_space(1)))* gcptr;
typedef const d4 __attribute__((address_space(1)))* gcptr4;

// Global-memory loads (the pointers come from descriptor tables, so the compiler would
// otherwise emit flat loads).
__device__ __forceinline__ double ldg(const double* p, int64_t i) { return ((gcptr)p)[i]; }
__device__ __forceinline__ d4 ldg4(const double* p) { return *((gcptr4)p); }

struct Frag {
    d4 a[2];   // a[i][t]: rows 16 i + r, K index 4 g + t
    d4 b[2];   // b[j][t]: columns 16 j + r, K index 4 g + t
};

__device__ __forceinline__ void mma_chunk(d4 (&acc)[2][2], const Frag& f) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < 2; ++nj)
                acc[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[mi][t], f.b[nj][t],
                                                                   acc[mi][nj], 0, 0, 0);
}

// Runs chunks c0, c0 + step, ... (< nch) with two register buffers: the loads of the next
// chunk are in flight while the MFMAs of the current one issue.
template <class Load>
__device__ __forceinline__ void kloop(d4 (&acc)[2][2], int c0, int step, int nch, Load load) {
    if (c0 >= nch) return;
    Frag f0, f1;
    int c = c0;
    load(c, f0);
    while (true) {
        const bool more = c + step < nch;
        if (more) load(c + step, f1);
        mma_chunk(acc, f0);
        if (!more) break;
        c += step;
        const bool more2 = c + step < nch;
        if (more2) load(c + step, f0);
        mma_chunk(acc, f1);
        if (!more2) break;
        c += step;
    }
}

__device__ __forceinline__ void zero_acc(d4 (&acc)[2][2]) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = (d4){0.0, 0.0, 0.0, 0.0};
}

__device__ __forceinline__ void scale_acc(d4 (&acc)[2][2], double s) {
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) acc[mi][nj] *= s;
}

// Stage 1: the K depth is one E-sector dimension (often below 16), so each wavefront owns a
// whole 32 x 64 tile (four tiles per work group, no split-K): the 32 rows of X it loads per
// chunk feed four 16-column panels of R, and the accumulators are stored directly.
__global__ __launch_bounds__(256, 2) void stage1_f64(const S1Block* __restrict__ blks,
                                                  const Tile* __restrict__ tiles, int ntiles,
                                                  const ProbPtrs* __restrict__ probs,
                                                  ProbPtrs single) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int ti = blockIdx.x * kWaves + wave;
    if (ti >= ntiles) return;
    const Tile tl = tiles[ti];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const S1Block B = blks[tl.blk];
    const ProbPtrs P = probs ? probs[B.prob] : single;
    if (P.skip && *P.skip) return;
    const int g = lane >> 4, r = lane & 15;
    const double xs = P.xscale ? *P.xscale : 1.0;
    const double* __restrict__ X = P.x;
    const int K = B.K, nch = B.nch;
    constexpr int NJ = kTile1N / 16;

    int64_t arow[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = min(tl.m0 + 16 * i + r, B.M - 1);
        const int pl = m >= B.X.split;
        arow[i] = B.X.off + pl * B.X.poff + (m - pl * B.X.split);
    }
    const double* pb = static_cast<const double*>(P.Rops) + B.Roff +
                       (((int64_t)(tl.n0 / kPanel) * nch) * 4 + g) * (kPanel * 4) + r * 4;
    const int64_t panel = (int64_t)nch * kChunkElems;   // doubles per packed column panel
    const int64_t ldx = B.X.ld;
    d4 acc[2][NJ];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) acc[mi][nj] = (d4){0.0, 0.0, 0.0, 0.0};
    d4 a[2][2], b[2][NJ];
    auto load = [&](int c, d4 (&fa)[2], d4 (&fb)[NJ]) {
        const int kb = c * kChunk + 4 * g;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int kk = min(kb + t, K - 1);
#pragma unroll
            for (int i = 0; i < 2; ++i) fa[i][t] = ldg(X, arow[i] + kk * ldx);
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) fb[j] = ldg4(pb + j * panel + (int64_t)c * kChunkElems);
    };
    auto mma = [&](const d4 (&fa)[2], const d4 (&fb)[NJ]) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int nj = 0; nj < NJ; ++nj)
                    acc[mi][nj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[mi][t], fb[nj][t],
                                                                       acc[mi][nj], 0, 0, 0);
    };
    load(0, a[0], b[0]);
    for (int c = 0;;) {
        const bool more = c + 1 < nch;
        if (more) load(c + 1, a[1], b[1]);
        mma(a[0], b[0]);
        if (!more) break;
        ++c;
        const bool more2 = c + 1 < nch;
        if (more2) load(c + 1, a[0], b[0]);
        mma(a[1], b[1]);
        if (!more2) break;
        ++c;
    }
    double* __restrict__ T = P.T;
    const View tv = B.T;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) {
            const int n = tl.n0 + 16 * nj + r;
            if (n >= B.N) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {   // f64 16x16 MFMA result: row g + 4v, column r
                const int m = tl.m0 + 16 * mi + g + 4 * v;
                if (m < B.M) {
                    const int pl = m >= tv.split;
                    T[tv.off + pl * tv.poff + (int64_t)n * tv.ld + (m - pl * tv.split)] =
                        acc[mi][nj][v] * xs;
                }
            }
        }
}

__global__ __launch_bounds__(256) void stage2_f64(const S2Block* __restrict__ blks,
                                                  const Segment* __restrict__ segs,
                                                  const Tile* __restrict__ tiles,
                                                  const ProbPtrs* __restrict__ probs,
                                                  ProbPtrs single) {
    const Tile tl = tiles[blockIdx.x];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const S2Block B = blks[tl.blk];
    const ProbPtrs P = probs ? probs[B.prob] : single;
    if (P.skip && *P.skip) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int g = lane >> 4, r = lane & 15;
    const double xs = P.xscale ? *P.xscale : 1.0;
    const int split = B.Y.split;   // columns per plane of the output and of every source

    const double* pa[2];
    int pl[2], col[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int pnl = tl.m0 / kPanel + i;
        pa[i] = static_cast<const double*>(P.Lops) + B.Aoff +
                (((int64_t)pnl * B.nch) * 4 + g) * (kPanel * 4) + r * 4;
        const int n = min(tl.n0 + 16 * i + r, B.N - 1);
        pl[i] = n >= split;
        col[i] = n - pl[i] * split;
    }
    d4 acc[2][2];
    zero_acc(acc);
    for (int s = 0; s < B.nseg; ++s) {
        const Segment sg = segs[B.seg0 + s];
        const double* __restrict__ src = sg.src ? P.T : P.x;
        int64_t bcol[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            bcol[i] = sg.B.off + pl[i] * sg.B.poff + (int64_t)col[i] * sg.B.ld;
        const int K = sg.K;
        auto load = [&](int c, Frag& f) {
            const int64_t ga = (int64_t)(sg.ch0 + c) * kChunkElems;
#pragma unroll
            for (int i = 0; i < 2; ++i) f.a[i] = ldg4(pa[i] + ga);
            const int kb = c * kChunk + 4 * g;
            if ((c + 1) * kChunk <= K) {   // full chunk: four consecutive doubles per lane
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int i = 0; i < 2; ++i) f.b[i][t] = ldg(src, bcol[i] + kb + t);
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int kk = min(kb + t, K - 1);
#pragma unroll
                    for (int i = 0; i < 2; ++i) f.b[i][t] = ldg(src, bcol[i] + kk);
                }
            }
        };
        const int nch = (K + kChunk - 1) / kChunk;
        // chunk c of this segment is global chunk ch0 + c, owned by wave (ch0 + c) mod 4
        const int c0 = ((wave - sg.ch0) % kWaves + kWaves) % kWaves;
        kloop(acc, c0, kWaves, nch, load);
        // segment 0 (the diagonal H_S term) is the only one reading the input vector: its
        // scale is applied to the accumulators before any other segment adds in
        if (s == 0) scale_acc(acc, xs);
    }

    __shared__ double red[kWaves][kTile][kTile + 1];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int v = 0; v < 4; ++v)   // f64 16x16 MFMA result: row g + 4v, column r
                red[wave][16 * nj + r][16 * mi + g + 4 * v] = acc[mi][nj][v];
    __syncthreads();
    const double* __restrict__ T = P.T;
    double* __restrict__ Y = P.y;
    const View t0 = B.T0, yv = B.Y;
    const int m = threadIdx.x & 31;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = (threadIdx.x >> 5) + 8 * q;
        const int gm = tl.m0 + m, gn = tl.n0 + n;
        if (gm < B.M && gn < B.N) {
            const double v = ((red[0][n][m] + red[1][n][m]) + red[2][n][m]) + red[3][n][m];
            const int p = gn >= split;
            const int c = gn - p * split;
            const double init = T[t0.off + p * t0.poff + (int64_t)c * t0.ld + gm];
            Y[yv.off + p * yv.poff + (int64_t)c * yv.ld + gm] = init + v;
        }
    }
}

hipError_t launch_stage1_f64(const S1Block* blks, const Tile* tiles, int ntiles,
                             const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    const int nblk = (ntiles + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(stage1_f64, dim3(nblk), dim3(256), 0, st, blks, tiles, ntiles, probs,
                       single);
    return hipGetLastError();
}

hipError_t launch_stage2_f64(const S2Block* blks, const Segment* segs, const Tile* tiles,
                             int ntiles, const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(stage2_f64, dim3(ntiles), dim3(256), 0, st, blks, segs, tiles, probs,
                       single);
    return hipGetLastError();
}

}  // namespace dmrg
