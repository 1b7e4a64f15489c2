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
// Stage 1 gives each wavefront its own 32 x 64 tile.  In stage 2 a work group of four
// wavefronts owns one 32 x 32 tile and deals its K chunks round-robin to the waves; the four
// partial tiles are summed in LDS in a fixed order (deterministic, no atomics).
//
// Inside one MFMA the K index each lane group supplies is free as long as A and B agree, so
// lane group g takes the KPL consecutive indices k = KPL g + t of a chunk.  The operator
// factors are packed in exactly that order (see internal.hpp), so lane (g, r) reads its part
// of a chunk as one contiguous piece, and they are zero-padded so no operator load needs a
// bounds check.  The data operands are read in place: rows (stage 1) or columns (stage 2) are
// contiguous in K.  The stage-1 workspace is zero-padded to whole chunks; for the input vector
// out-of-range K indices are clamped to a valid element, whose product with the padded zeros
// vanishes.
#include "internal.hpp"

namespace dmrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Global-memory loads (pointers from descriptor tables would otherwise become flat loads).
template <typename T>
__device__ __forceinline__ T ldg(const T* p, int64_t i) {
    return ((const __attribute__((address_space(1))) T*)p)[i];
}
template <typename V>
__device__ __forceinline__ V ldgv(const void* p) {
    return *((const __attribute__((address_space(1))) V*)p);
}

// ---------------------------------------------------------------------------------------
// arithmetic traits
// ---------------------------------------------------------------------------------------
struct PF64 {
    static constexpr int CK = 16, KPL = 4, PER = 1;   // PER: packed pieces per value
    using op_t = double;          // packed operator element
    using ws_t = double;          // workspace element
    using acc_t = d4;
    using frag_t = d4;            // one lane's operand values of one chunk
    __device__ static frag_t from(const double (&v)[KPL]) { return (d4){v[0], v[1], v[2], v[3]}; }
    __device__ static frag_t load_op(const op_t* p) { return ldgv<d4>(p); }
    __device__ static acc_t mma(const frag_t& a, const frag_t& b, acc_t c) {
#pragma unroll
        for (int t = 0; t < 4; ++t) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], c, 0, 0, 0);
        return c;
    }
    __device__ static int row(int g, int v) { return g + 4 * v; }   // result lane layout
};

struct PF32 {
    static constexpr int CK = 16, KPL = 4, PER = 1;
    using op_t = float;
    using ws_t = float;
    using acc_t = f4;
    using frag_t = f4;
    __device__ static frag_t from(const double (&v)[KPL]) {
        return (f4){(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    }
    __device__ static frag_t load_op(const op_t* p) { return ldgv<f4>(p); }
    __device__ static acc_t mma(const frag_t& a, const frag_t& b, acc_t c) {
#pragma unroll
        for (int t = 0; t < 4; ++t) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[t], c, 0, 0, 0);
        return c;
    }
    __device__ static int row(int g, int v) { return 4 * g + v; }
};

// Split bf16 operands: NP pieces per value; the products of total order below NP (pieces
// i + j < NP) are accumulated, smallest orders last.
template <int NP>
struct PSplit {
    static constexpr int CK = 32, KPL = 8, PER = NP;
    using op_t = __bf16;          // packed as KPL values of piece 0, then piece 1, ... per lane
    using ws_t = float;
    using acc_t = f4;
    struct frag_t {
        bf8 p[NP];
    };
    __device__ static frag_t from(const double (&v)[KPL]) {
        frag_t f;
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
            float rest = (float)v[t];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const __bf16 h = (__bf16)rest;
                f.p[q][t] = h;
                rest -= (float)h;
            }
        }
        return f;
    }
    __device__ static frag_t load_op(const op_t* p) {
        frag_t f;
#pragma unroll
        for (int q = 0; q < NP; ++q) f.p[q] = ldgv<bf8>(p + q * KPL);
        return f;
    }
    __device__ static acc_t mma(const frag_t& a, const frag_t& b, acc_t c) {
#pragma unroll
        for (int o = 0; o < NP; ++o)
#pragma unroll
            for (int i = 0; i <= o; ++i)
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[i], b.p[o - i], c, 0, 0, 0);
        return c;
    }
    __device__ static int row(int g, int v) { return 4 * g + v; }
};
using PBF3 = PSplit<2>;
using PBF6 = PSplit<3>;

// Elements of one packed panel chunk per lane (all pieces of a split value) and per chunk.
template <class P>
constexpr int lane_elems() {
    return P::KPL * P::PER;
}
template <class P>
constexpr int chunk_elems() {
    return kPanel * 4 * lane_elems<P>();
}

template <class P>
__device__ __forceinline__ void zero(typename P::acc_t& a) {
#pragma unroll
    for (int v = 0; v < 4; ++v) a[v] = 0;
}

// KPL consecutive data values v[t] = src[base + t] (workspace, zero-padded chunks)
template <class P, typename T>
__device__ __forceinline__ void load_run(const T* src, int64_t base, double (&v)[P::KPL]) {
#pragma unroll
    for (int t = 0; t < P::KPL; ++t) v[t] = (double)ldg(src, base + t);
}
// KPL values src[base + min(k0 + t, K - 1) * stride] (input vector, clamped)
template <class P>
__device__ __forceinline__ void load_clamped(const double* src, int64_t base, int k0, int K,
                                             int64_t stride, double (&v)[P::KPL]) {
#pragma unroll
    for (int t = 0; t < P::KPL; ++t) v[t] = ldg(src, base + (int64_t)min(k0 + t, K - 1) * stride);
}

// ---------------------------------------------------------------------------------------
// stage 1: one 32 x 64 tile per wavefront
// ---------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(256, 2) void stage1(const S1Block* __restrict__ blks,
                                                 const Tile* __restrict__ tiles, int ntiles,
                                                 const ProbPtrs* __restrict__ probs,
                                                 ProbPtrs single) {
    using op_t = typename P::op_t;
    using ws_t = typename P::ws_t;
    using acc_t = typename P::acc_t;
    using frag_t = typename P::frag_t;
    constexpr int NJ = kTile1N / 16;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int ti = blockIdx.x * kWaves + wave;
    if (ti >= ntiles) return;
    const Tile tl = tiles[ti];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const S1Block B = blks[tl.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    const int g = lane >> 4, r = lane & 15;
    const double xs = P_.xscale ? *P_.xscale : 1.0;
    const double* __restrict__ X = P_.x;
    const int K = B.K;
    const int nch = (K + P::CK - 1) / P::CK;

    int64_t arow[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int m = min(tl.m0 + 16 * i + r, B.M - 1);
        const int pl = m >= B.X.split;
        arow[i] = B.X.off + pl * B.X.poff + (m - pl * B.X.split);
    }
    const op_t* pb = static_cast<const op_t*>(P_.Rops) + B.Roff * P::PER +
                     (((int64_t)(tl.n0 / kPanel) * nch) * 4 + g) * (kPanel * lane_elems<P>()) +
                     r * lane_elems<P>();
    const int64_t panel = (int64_t)nch * chunk_elems<P>();
    const int64_t ldx = B.X.ld;
    acc_t acc[2][NJ];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) zero<P>(acc[mi][nj]);
    frag_t a[2][2], b[2][NJ];
    auto load = [&](int c, frag_t (&fa)[2], frag_t (&fb)[NJ]) {
        const int kb = c * P::CK + P::KPL * g;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            double v[P::KPL];
            load_clamped<P>(X, arow[i], kb, K, ldx, v);
            fa[i] = P::from(v);
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) fb[j] = P::load_op(pb + j * panel + (int64_t)c * chunk_elems<P>());
    };
    auto mma = [&](const frag_t (&fa)[2], const frag_t (&fb)[NJ]) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < NJ; ++nj) acc[mi][nj] = P::mma(fa[mi], fb[nj], acc[mi][nj]);
    };
    // two register buffers; the prefetch is unconditional (chunk index clamped) so that no
    // load sits under a branch and the compiler waits only for the buffer being consumed
    load(0, a[0], b[0]);
    for (int c = 0;; c += 2) {
        load(min(c + 1, nch - 1), a[1], b[1]);
        mma(a[0], b[0]);
        if (c + 1 >= nch) break;
        load(min(c + 2, nch - 1), a[0], b[0]);
        mma(a[1], b[1]);
        if (c + 2 >= nch) break;
    }
    ws_t* __restrict__ T = static_cast<ws_t*>(P_.T);
    const View tv = B.T;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
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
                        (ws_t)(acc[mi][nj][v] * xs);
                }
            }
        }
}

// ---------------------------------------------------------------------------------------
// stage 2: one 32 x 32 tile per work group, K chunks dealt round-robin to the four waves
// ---------------------------------------------------------------------------------------
template <class P, class Load>
__device__ __forceinline__ void kloop(typename P::acc_t (&acc)[2][2], int c0, int step, int nch,
                                      Load load) {
    using frag_t = typename P::frag_t;
    if (c0 >= nch) return;
    const int last = c0 + (nch - 1 - c0) / step * step;
    frag_t a0[2], b0[2], a1[2], b1[2];
    auto mma = [&](const frag_t (&fa)[2], const frag_t (&fb)[2]) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = P::mma(fa[mi], fb[nj], acc[mi][nj]);
    };
    // unconditional (clamped) prefetch, as in stage 1
    load(c0, a0, b0);
    for (int c = c0;; c += 2 * step) {
        load(min(c + step, last), a1, b1);
        mma(a0, b0);
        if (c + step > last) break;
        load(min(c + 2 * step, last), a0, b0);
        mma(a1, b1);
        if (c + 2 * step > last) break;
    }
}

template <class P>
__global__ __launch_bounds__(256, 3) void stage2(const S2Block* __restrict__ blks,
                                                 const Segment* __restrict__ segs,
                                                 const Tile* __restrict__ tiles,
                                                 const ProbPtrs* __restrict__ probs,
                                                 ProbPtrs single) {
    using op_t = typename P::op_t;
    using ws_t = typename P::ws_t;
    using acc_t = typename P::acc_t;
    using frag_t = typename P::frag_t;
    const Tile tl = tiles[blockIdx.x];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const S2Block B = blks[tl.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int g = lane >> 4, r = lane & 15;
    const double xs = P_.xscale ? *P_.xscale : 1.0;
    const int split = B.Y.split;   // columns per plane of the output and of every source
    const ws_t* __restrict__ Tws = static_cast<const ws_t*>(P_.T);

    const op_t* pa[2];
    int pl[2], col[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int pnl = tl.m0 / kPanel + i;
        pa[i] = static_cast<const op_t*>(P_.Lops) + B.Aoff * P::PER +
                (((int64_t)pnl * B.nch) * 4 + g) * (kPanel * lane_elems<P>()) + r * lane_elems<P>();
        const int n = min(tl.n0 + 16 * i + r, B.N - 1);
        pl[i] = n >= split;
        col[i] = n - pl[i] * split;
    }
    acc_t acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) zero<P>(acc[mi][nj]);
    for (int s = 0; s < B.nseg; ++s) {
        const Segment sg = segs[B.seg0 + s];
        int64_t bcol[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            bcol[i] = sg.B.off + pl[i] * sg.B.poff + (int64_t)col[i] * sg.B.ld;
        const int K = sg.K;
        const int nch = (K + P::CK - 1) / P::CK;
        // chunk c of this segment is global chunk ch0 + c, owned by wave (ch0 + c) mod 4
        const int c0 = ((wave - sg.ch0) % kWaves + kWaves) % kWaves;
        if (sg.src) {
            auto load = [&](int c, frag_t (&fa)[2], frag_t (&fb)[2]) {
                const int64_t ga = (int64_t)(sg.ch0 + c) * chunk_elems<P>();
#pragma unroll
                for (int i = 0; i < 2; ++i) fa[i] = P::load_op(pa[i] + ga);
                const int kb = c * P::CK + P::KPL * g;
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    double v[P::KPL];
                    load_run<P>(Tws, bcol[i] + kb, v);
                    fb[i] = P::from(v);
                }
            };
            kloop<P>(acc, c0, kWaves, nch, load);
        } else {
            auto load = [&](int c, frag_t (&fa)[2], frag_t (&fb)[2]) {
                const int64_t ga = (int64_t)(sg.ch0 + c) * chunk_elems<P>();
#pragma unroll
                for (int i = 0; i < 2; ++i) fa[i] = P::load_op(pa[i] + ga);
                const int kb = c * P::CK + P::KPL * g;
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    double v[P::KPL];
                    load_clamped<P>(P_.x, bcol[i], kb, K, 1, v);
                    fb[i] = P::from(v);
                }
            };
            kloop<P>(acc, c0, kWaves, nch, load);
            // segment 0 (the diagonal H_S term) is the only one reading the input vector:
            // its scale is applied before any other segment adds in
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int nj = 0; nj < 2; ++nj)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[mi][nj][v] *= xs;
        }
    }

    __shared__ double red[kWaves][kTile][kTile + 1];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                red[wave][16 * nj + r][16 * mi + P::row(g, v)] = (double)acc[mi][nj][v];
    __syncthreads();
    double* __restrict__ Y = P_.y;
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
            const double init = (double)Tws[t0.off + p * t0.poff + (int64_t)c * t0.ld + gm];
            Y[yv.off + p * yv.poff + (int64_t)c * yv.ld + gm] = init + v;
        }
    }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
namespace {

template <class P>
hipError_t launch1(const S1Block* blks, const Tile* tiles, int ntiles, const ProbPtrs* probs,
                   ProbPtrs single, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    const int nblk = (ntiles + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(stage1<P>, dim3(nblk), dim3(256), 0, st, blks, tiles, ntiles, probs, single);
    return hipGetLastError();
}

template <class P>
hipError_t launch2(const S2Block* blks, const Segment* segs, const Tile* tiles, int ntiles,
                   const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(stage2<P>, dim3(ntiles), dim3(256), 0, st, blks, segs, tiles, probs, single);
    return hipGetLastError();
}

}  // namespace

// prec: 0 FP64, 1 FP32, 2 BF16x3, 3 BF16x6 (the operator buffers and workspace must match)
hipError_t launch_stage1(int prec, const S1Block* blks, const Tile* tiles, int ntiles,
                         const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    switch (prec) {
        case 0: return launch1<PF64>(blks, tiles, ntiles, probs, single, st);
        case 1: return launch1<PF32>(blks, tiles, ntiles, probs, single, st);
        case 2: return launch1<PBF3>(blks, tiles, ntiles, probs, single, st);
        default: return launch1<PBF6>(blks, tiles, ntiles, probs, single, st);
    }
}

hipError_t launch_stage2(int prec, const S2Block* blks, const Segment* segs, const Tile* tiles,
                         int ntiles, const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    switch (prec) {
        case 0: return launch2<PF64>(blks, segs, tiles, ntiles, probs, single, st);
        case 1: return launch2<PF32>(blks, segs, tiles, ntiles, probs, single, st);
        case 2: return launch2<PBF3>(blks, segs, tiles, ntiles, probs, single, st);
        default: return launch2<PBF6>(blks, segs, tiles, ntiles, probs, single, st);
    }
}

}  // namespace dmrg
