// Grouped block products of H_sb.psi on gfx950 FP64 MFMA (v_mfma_f64_16x16x4f64).
//
// The Hamiltonian connections (Sec. IV) are applied as psi' = A psi B^T over (N_up, N_dn)
// symmetry blocks in two stages, each one launch over a list of 32 x 32 output tiles:
//   stage 1  T_b  = X_b R_b        right products, X_b = [Re; Im] planes of the source block
//   stage 2  Y_b' = T0 + Acat Bcat left products summed over all terms entering the block
// A work group of four wavefronts owns one tile and splits its K range into 16-deep chunks
// dealt round-robin to the waves; the four partial tiles are summed in LDS in a fixed order
// (deterministic, no atomics).  Each wave holds 2 x 2 MFMA accumulators (32 x 32).
//
// Operand loads go straight from global memory into the MFMA input registers: inside one
// 4-deep MFMA step the K index each lane group supplies is free as long as A and B agree, so
// lane group g takes k = 4g + t at step t.  A operands (row-contiguous) are then read as four
// 128-byte column pieces per instruction, B operands (K-contiguous) as four consecutive
// doubles per lane.
#include "internal.hpp"

namespace dmrg {

typedef double d4 __attribute__((ext_vector_type(4)));

struct Frag {
    double a[2][4];
    double b[2][4];
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

// Sums the four waves' partial tiles; calls out(m, n, value) for every in-range element.
template <typename Out>
__device__ __forceinline__ void reduce_tile(const d4 (&acc)[2][2], int M, int N, int m0, int n0,
                                            Out out) {
    __shared__ double red[kWaves][kTile][kTile + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int v = 0; v < 4; ++v)   // f64 16x16 MFMA result: row g + 4v, column r
                red[wave][16 * nj + r][16 * mi + g + 4 * v] = acc[mi][nj][v];
    __syncthreads();
    const int m = threadIdx.x & 31;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int n = (threadIdx.x >> 5) + 8 * q;
        if (m0 + m < M && n0 + n < N) {
            const double s = ((red[0][n][m] + red[1][n][m]) + red[2][n][m]) + red[3][n][m];
            out(m0 + m, n0 + n, s);
        }
    }
}

__global__ __launch_bounds__(256) void stage1_f64(const S1Block* __restrict__ blks,
                                                  const Tile* __restrict__ tiles,
                                                  const ProbPtrs* __restrict__ probs,
                                                  ProbPtrs single) {
    const Tile tl = tiles[blockIdx.x];
    const S1Block B = blks[tl.blk];
    const ProbPtrs P = probs ? probs[B.prob] : single;
    if (P.skip && *P.skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const double xs = P.xscale ? *P.xscale : 1.0;
    const double* __restrict__ X = P.x;
    const double* __restrict__ R = static_cast<const double*>(P.Rops) + B.Roff;

    int64_t arow[2], bcol[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = min(tl.m0 + 16 * i + r, B.M - 1);
        const int pl = m >= B.X.split;
        arow[i] = B.X.off + pl * B.X.poff + (m - pl * B.X.split);
        const int n = min(tl.n0 + 16 * i + r, B.N - 1);
        bcol[i] = (int64_t)n * B.K;
    }
    const int64_t ldx = B.X.ld;
    const int K = B.K;
    auto load = [&](int ch, Frag& f) {
        const int kb = ch * kChunk + 4 * g;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = kb + t;
            const bool ok = k < K;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                f.a[i][t] = ok ? X[arow[i] + k * ldx] * xs : 0.0;
                f.b[i][t] = ok ? R[bcol[i] + k] : 0.0;
            }
        }
    };
    d4 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = (d4){0.0, 0.0, 0.0, 0.0};
    const int nch = (K + kChunk - 1) / kChunk;
    int ch = wave;
    if (ch < nch) {
        Frag cur, nxt;
        load(ch, cur);
        for (; ch + kWaves < nch; ch += kWaves) {
            load(ch + kWaves, nxt);
            mma_chunk(acc, cur);
            cur = nxt;
        }
        mma_chunk(acc, cur);
    }
    double* __restrict__ T = P.T + B.Toff;
    const int M = B.M;
    reduce_tile(acc, B.M, B.N, tl.m0, tl.n0,
                [&](int m, int n, double v) { T[(int64_t)n * M + m] = v; });
}

__global__ __launch_bounds__(256) void stage2_f64(const S2Block* __restrict__ blks,
                                                  const Segment* __restrict__ segs,
                                                  const Tile* __restrict__ tiles,
                                                  const ProbPtrs* __restrict__ probs,
                                                  ProbPtrs single) {
    const Tile tl = tiles[blockIdx.x];
    const S2Block B = blks[tl.blk];
    const ProbPtrs P = probs ? probs[B.prob] : single;
    if (P.skip && *P.skip) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const double xs = P.xscale ? *P.xscale : 1.0;
    const double* __restrict__ A = static_cast<const double*>(P.Lops) + B.Aoff;
    const int M = B.M;
    const int split = B.Y.split;   // columns per plane of the output and of every source

    int arow[2], pl[2], col[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        arow[i] = min(tl.m0 + 16 * i + r, M - 1);
        const int n = min(tl.n0 + 16 * i + r, B.N - 1);
        pl[i] = n >= split;
        col[i] = n - pl[i] * split;
    }
    d4 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = (d4){0.0, 0.0, 0.0, 0.0};

    int gc = 0;   // chunks dealt so far (round-robin over the waves across segments)
    for (int s = 0; s < B.nseg; ++s) {
        const Segment sg = segs[B.seg0 + s];
        const double* __restrict__ src = sg.src ? P.T : P.x;
        const double sc = sg.src ? 1.0 : xs;
        int64_t bcol[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) bcol[i] = sg.B.off + pl[i] * sg.B.poff + (int64_t)col[i] * sg.B.ld;
        const int K = sg.K;
        const double* __restrict__ As = A + (int64_t)sg.kA * M;
        auto load = [&](int ch, Frag& f) {
            const int kb = ch * kChunk + 4 * g;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = kb + t;
                const bool ok = k < K;
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    f.a[i][t] = ok ? As[(int64_t)k * M + arow[i]] : 0.0;
                    f.b[i][t] = ok ? src[bcol[i] + k] * sc : 0.0;
                }
            }
        };
        const int nch = (K + kChunk - 1) / kChunk;
        int ch = ((wave - gc) % kWaves + kWaves) % kWaves;
        gc += nch;
        if (ch >= nch) continue;
        Frag cur, nxt;
        load(ch, cur);
        for (; ch + kWaves < nch; ch += kWaves) {
            load(ch + kWaves, nxt);
            mma_chunk(acc, cur);
            cur = nxt;
        }
        mma_chunk(acc, cur);
    }
    const double* __restrict__ T = P.T;
    double* __restrict__ Y = P.y;
    const View t0 = B.T0, yv = B.Y;
    reduce_tile(acc, B.M, B.N, tl.m0, tl.n0, [&](int m, int n, double v) {
        const int p = n >= split;
        const int c = n - p * split;
        const double init = T[t0.off + p * t0.poff + (int64_t)c * t0.ld + m];
        Y[yv.off + p * yv.poff + (int64_t)c * yv.ld + m] = init + v;
    });
}

hipError_t launch_stage1_f64(const S1Block* blks, const Tile* tiles, int ntiles,
                             const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(stage1_f64, dim3(ntiles), dim3(256), 0, st, blks, tiles, probs, single);
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
