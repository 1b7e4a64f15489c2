// K-split FP64 block products of H_sb.psi on gfx950 (the work lists and layouts are described
// with KPack in internal.hpp).
//
// Why: measured on this part, v_mfma_f64_16x16x4f64 sustains about 44 TFLOP/s, while
// v_mfma_f64_4x4x4_4b_f64 sustains about 69 TFLOP/s.  The 4x4x4 form (four blocks) takes, in
// lane l = 16 k' + 4 b + x, A(row x, k') and B(k', column x) of block b, and returns D(row t,
// column j) of block b in lane 16 t + 4 b + j.  Taking the four blocks as four slices of a
// 16-deep K chunk (k = 4 b + k'), one instruction multiplies a 4 x 16 piece of A by a 16 x 4
// piece of B into four partial 4 x 4 products, which are added across the lane groups b once
// per tile.  No operand is broadcast, so both can come straight from memory, packed in lane
// order: 16-byte loads of whole 1 KB runs, no LDS staging.  A wavefront's 32 x 32 tile holds 64
// accumulators (one double per lane each) and loads 8 KB per chunk for 64 instructions.
//
// Tiles at block edges cover 16, 8 or 4 rows (columns) with their own instantiations, so the
// flops spent on padding are those of whole groups of 4 (not of 16 or 32).
#include <hip/hip_runtime.h>

#include "mfma.hpp"

namespace dmrg {

namespace {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef double dd2 __attribute__((ext_vector_type(2)));

// DPP move of a double within rows of 16 lanes (row rotation by CTRL - 0x120 lanes).
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the four K slices b (lanes 16 t + 4 b + j, t and j fixed): rotations by 4 and 8
// lanes within each row of 16 lanes; every lane gets the sum of its (t, j).
__device__ __forceinline__ double ksum(double v) {
    v += dppd<0x124>(v);
    v += dppd<0x128>(v);
    return v;
}

// Operand values of one chunk: N groups (1, 2, 4 or 8) from pairs of a packed piece.
// p: element (pair i0, lane, s0) of chunk 0; step: elements per chunk.
template <int N>
struct Ops {
    double v[N];
    __device__ __forceinline__ void load(const double* p) {
        if constexpr (N == 1) {
            v[0] = ldg(p, 0);
        } else {
#pragma unroll
            for (int i = 0; i < N / 2; ++i) {
                const dd2 w = ldgv<dd2>(p + i * 128);
                v[2 * i] = w.x;
                v[2 * i + 1] = w.y;
            }
        }
    }
};

template <int RQ, int CP>
__device__ __forceinline__ void mma(double (&acc)[RQ][CP], const Ops<RQ>& a, const Ops<CP>& b) {
#pragma unroll
    for (int q = 0; q < RQ; ++q)
#pragma unroll
        for (int p = 0; p < CP; ++p)
            acc[q][p] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.v[q], b.v[p], acc[q][p], 0, 0, 0);
}

// Register sets of operands in flight for a tile shape: what the accumulators leave of a budget
// of 120 doubles, 2 to 8 sets.  Thin tiles do few products per chunk, so they need more chunks
// in flight to cover the latency of their loads.
template <int RQ, int CP>
constexpr int ksets() {
    const int n = (120 - RQ * CP) / (RQ + CP);
    return n < 2 ? 2 : (n > 8 ? 8 : n);
}

// Chunks c0, c0 + step, ..., <= last through NS rotating register sets: while set s is
// multiplied, the next NS - 1 chunks' loads are in flight.  Every step issues the loads of
// exactly one set (chunks past the last are loaded clamped, harmless, never multiplied), so the
// wait before each product counts exactly the newer loads.
// pa(c), pb(c): the operands' element pointers for chunk c.
template <int RQ, int CP, class PA, class PB>
__device__ __forceinline__ void kloop(double (&acc)[RQ][CP], int c0, int last, int step, PA&& pa,
                                      PB&& pb) {
    constexpr int NS = ksets<RQ, CP>();
    if (c0 > last) return;
    Ops<RQ> a[NS];
    Ops<CP> b[NS];
    // Drain whatever the caller left in flight: several shapes share one kernel, and without
    // this the wait at the head of every shape's loop merges the other shapes' loads into a
    // full drain per round.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) {
        const int cs = min(c0 + s * step, last);
        a[s].load(pa(cs));
        b[s].load(pb(cs));
    }
    // whole rounds of NS chunks (no condition inside, exact waits); at the start of a round set
    // s holds chunk c + s step for s < NS - 1
    int c = c0;
    for (; c + (NS - 1) * step <= last; c += NS * step) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int cl = min(c + (s + NS - 1) * step, last);
            a[(s + NS - 1) % NS].load(pa(cl));
            b[(s + NS - 1) % NS].load(pb(cl));
            __builtin_amdgcn_sched_barrier(0);
            mma(acc, a[s], b[s]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // the last chunks (fewer than NS - 1), already in sets 0 ..
#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
        if (c + s * step <= last) mma(acc, a[s], b[s]);
}

// Element pointer of groups g0.. of chunk 0 in a packed operand (lane's own element).
__device__ __forceinline__ int64_t kbase(const KPack& pk, int g0, int lane, int n) {
    return pk.off + (int64_t)(g0 / 8) * pk.pstride * kKPiece + ((g0 % 8) / 2) * 128 + lane * 2 +
           (n == 1 ? (g0 & 1) : 0);
}

// ---------------------------------------------------------------------------------------
// pre-pack of the input vector: one piece per work group of one wavefront
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_prepack(const KXBlock* __restrict__ blks,
                                                const KPItem* __restrict__ items,
                                                const ProbPtrs* __restrict__ probs,
                                                ProbPtrs single) {
    const KPItem it = items[blockIdx.x];
    if (it.blk < 0) return;
    const KXBlock B = blks[it.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    const int64_t np = B.xplane;
    const int lane = threadIdx.x;
    const int kq = lane >> 4, bq = (lane >> 2) & 3, x = lane & 3;
    const double* __restrict__ X = P_.x;
    const KPack pk = it.which == 0 ? B.xa : B.xb;
    double* out = static_cast<double*>(P_.T) + pk.off +
                  ((int64_t)it.P * pk.pstride + (int64_t)it.c * pk.cstride) * kKPiece + lane * 2;
    const int k = 16 * it.c + 4 * bq + kq;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double v[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int r = 32 * it.P + 4 * (2 * i + s) + x;
            double val = 0.0;
            if (it.which == 0) {          // X_b (2 dpad x e): row r = plane dpad + row, column k
                const int pl = r >= B.dpad, ri = r - pl * B.dpad;
                if (ri < B.d && k < B.e) val = ldg(X, B.xoff + pl * np + ri + (int64_t)k * B.d);
            } else {                      // the block as a B operand (d x 2 epad): row k, column r
                const int pl = r >= B.epad, rj = r - pl * B.epad;
                if (rj < B.e && k < B.d) val = ldg(X, B.xoff + pl * np + k + (int64_t)rj * B.d);
            }
            v[s] = val;
        }
        *reinterpret_cast<dd2*>(out + i * 128) = (dd2){v[0], v[1]};
    }
}

// ---------------------------------------------------------------------------------------
// stage 1: one tile per work group of one wavefront
// ---------------------------------------------------------------------------------------
template <int LQ, int LP>
__device__ __forceinline__ void s1_tile(const KTile& tl, const KS1Block& B,
                                        const KEdgeOut* __restrict__ eout, const ProbPtrs& P_) {
    constexpr int RQ = 1 << LQ, CP = 1 << LP;
    const int lane = threadIdx.x & 63;
    const double* __restrict__ W = static_cast<const double*>(P_.T);
    const double* __restrict__ R = static_cast<const double*>(P_.Rops);
    const double* pa0 = W + kbase(B.A, tl.g0, lane, RQ);
    const double* pb0 = R + kbase(B.B, tl.h0, lane, CP);
    const int64_t sa = (int64_t)B.A.cstride * kKPiece, sb = (int64_t)B.B.cstride * kKPiece;
    double acc[RQ][CP];
#pragma unroll
    for (int q = 0; q < RQ; ++q)
#pragma unroll
        for (int p = 0; p < CP; ++p) acc[q][p] = 0.0;
    kloop<RQ, CP>(acc, 0, B.nch - 1, 1, [&](int c) { return pa0 + c * sa; },
                  [&](int c) { return pb0 + c * sb; });
    // outputs: after the sum over the K slices, every lane (t, b, j) holds element (row
    // 4 (g0 + q) + t, column 4 (h0 + p) + j) of accumulator (q, p).  The tile lies in one plane
    // and one column segment.  Lane group b stores the accumulators of the row groups whose
    // position in their 16-row chunk is b (row group q: (g0r + q) mod 4 = b, g0r = the tile's
    // first row group within the plane), so that in the edge's packed operand every lane writes
    // its own lane slot: one contiguous run per store.
    const int t = lane >> 4, bq = (lane >> 2) & 3, j = lane & 3;
    double* __restrict__ T = static_cast<double*>(P_.T);
#pragma unroll
    for (int q = 0; q < RQ; ++q)
#pragma unroll
        for (int p = 0; p < CP; ++p) acc[q][p] = ksum(acc[q][p]);
    const int pl = tl.plane;
    const int g0r = tl.g0 - pl * (B.dpad / 4);                 // row groups within the plane
    constexpr int NQ = RQ < 4 ? 1 : RQ / 4;                    // row quads
    const int qo = (bq - g0r) & 3;                             // this lane's row group in a quad
    if (tl.seg < 0) {
        // T0 (d x 2 epad, column-major): rows i < d, columns jj < e of plane pl
        const int jj0 = 4 * tl.h0;
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
            const int qq = 4 * r + qo;
            if (RQ < 4 && qq >= RQ) continue;
            const int i = 4 * (g0r + qq) + t;
#pragma unroll
            for (int p = 0; p < CP; ++p) {
                double v = acc[4 * r][p];
#pragma unroll
                for (int u = 1; u < (RQ < 4 ? RQ : 4); ++u)
                    if (qo == u) v = acc[4 * r + u][p];
                const int jj = jj0 + 4 * p + j;
                if (i < B.d && jj < B.e)
                    T[B.t0off + (int64_t)(pl * B.epad + jj) * B.d + i] = v;
            }
        }
        return;
    }
    // an edge: element (k = i, column nn = pl e2pad + jj) of its packed stage-2 operand; rows of
    // the last chunk past d and columns past e2 receive exact zeros (zero pack rows and factor
    // columns), so they are stored unmasked
    const KEdgeOut eo = eout[B.edge0 + tl.seg];
    const int nn0 = pl * eo.e2pad + 4 * tl.h0 - eo.col;
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
        const int qq = 4 * r + qo;
        if (RQ < 4 && qq >= RQ) continue;
        const int i = 4 * (g0r + qq) + t;
        double* piece = T + eo.P.off + (int64_t)(i / 16) * eo.P.cstride * kKPiece + lane * 2;
        auto val = [&](int p) {
            double v = acc[4 * r][p];
#pragma unroll
            for (int u = 1; u < (RQ < 4 ? RQ : 4); ++u)
                if (qo == u) v = acc[4 * r + u][p];
            return v;
        };
        if constexpr (CP == 1) {
            const int nn = nn0, grp = (nn % kKPanel) / 4;
            piece[(int64_t)(nn / kKPanel) * eo.P.pstride * kKPiece + (grp / 2) * 128 + (grp & 1)] = val(0);
        } else {
#pragma unroll
            for (int p = 0; p < CP; p += 2) {
                const int nn = nn0 + 4 * p, grp = (nn % kKPanel) / 4;   // grp even: a pair
                *reinterpret_cast<dd2*>(piece + (int64_t)(nn / kKPanel) * eo.P.pstride * kKPiece +
                                        (grp / 2) * 128) = (dd2){val(p), val(p + 1)};
            }
        }
    }
}

__global__ __launch_bounds__(64, 2) void stage1k(const KS1Block* __restrict__ blks,
                                              const KEdgeOut* __restrict__ eout,
                                              const KTile* __restrict__ tiles,
                                              const ProbPtrs* __restrict__ probs, ProbPtrs single) {
    const KTile tl = tiles[blockIdx.x];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const KS1Block B = blks[tl.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    switch (tl.shape) {
#define DMRG_K1(Q, P) \
    case 4 * Q + P: s1_tile<Q, P>(tl, B, eout, P_); break;
        DMRG_K1(3, 3) DMRG_K1(3, 2) DMRG_K1(3, 1) DMRG_K1(3, 0)
        DMRG_K1(2, 3) DMRG_K1(2, 2) DMRG_K1(2, 1) DMRG_K1(2, 0)
        DMRG_K1(1, 3) DMRG_K1(1, 2) DMRG_K1(1, 1) DMRG_K1(1, 0)
        DMRG_K1(0, 3) DMRG_K1(0, 2) DMRG_K1(0, 1) DMRG_K1(0, 0)
#undef DMRG_K1
        default: break;
    }
}

// ---------------------------------------------------------------------------------------
// stage 2: one tile per work group of four wavefronts (K chunks dealt round-robin)
// ---------------------------------------------------------------------------------------
constexpr int kK2Threads = 256;

template <int LQ, int LP>
__device__ __forceinline__ void s2_tile(const KTile& tl, const KS2Block& B,
                                        const int64_t* __restrict__ ctab, const ProbPtrs& P_,
                                        double* __restrict__ part) {
    constexpr int RQ = 1 << LQ, CP = 1 << LP, NACC = RQ * CP;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double* __restrict__ W = static_cast<const double*>(P_.T);
    const double* __restrict__ Lf = static_cast<const double*>(P_.Lops);
    const double* pa0 = Lf + kbase(B.A, tl.g0, lane, RQ);
    const int64_t sa = (int64_t)B.A.cstride * kKPiece;
    // B: chunk c's piece of column panel 0 at W + ctab[c]; panels one piece apart
    const int64_t bo = (int64_t)(tl.h0 / 8) * kKPiece + ((tl.h0 % 8) / 2) * 128 + lane * 2 +
                       (CP == 1 ? (tl.h0 & 1) : 0);
    const int64_t* __restrict__ ct = ctab + B.ctab0;
    double acc[RQ][CP];
#pragma unroll
    for (int q = 0; q < RQ; ++q)
#pragma unroll
        for (int p = 0; p < CP; ++p) acc[q][p] = 0.0;
    kloop<RQ, CP>(acc, wave, B.nch - 1, 4, [&](int c) { return pa0 + c * sa; },
                  [&](int c) { return W + ct[c] + bo; });
#pragma unroll
    for (int q = 0; q < RQ; ++q)
#pragma unroll
        for (int p = 0; p < CP; ++p) acc[q][p] = ksum(acc[q][p]);
    // partial tiles of waves 1..3 through LDS: lane (t, b, j) writes the accumulators it owns
    // (index mod 4 = b), 16 distinct values per accumulator
    const int t = lane >> 4, bq = (lane >> 2) & 3, j = lane & 3;
    const int slot = 4 * t + j;   // output (t, j) of an accumulator
    if (wave > 0) {
#pragma unroll
        for (int q = 0; q < RQ; ++q)
#pragma unroll
            for (int p = 0; p < CP; ++p)
                if (((q * CP + p) & 3) == bq) part[((wave - 1) * NACC + q * CP + p) * 16 + slot] = acc[q][p];
    }
    __syncthreads();
    if (wave != 0) return;
    double* __restrict__ Y = P_.y;
    const View yv = B.Y;
#pragma unroll
    for (int q = 0; q < RQ; ++q)
#pragma unroll
        for (int p = 0; p < CP; ++p) {
            if (((q * CP + p) & 3) != bq) continue;
            const int m = 4 * (tl.g0 + q) + t, nn = 4 * (tl.h0 + p) + j;
            const int pl = nn >= B.epad, jn = nn - pl * B.epad;   // plane, column in the plane
            if (m >= B.M || jn >= B.e) continue;
            double v = acc[q][p];                      // fixed order: waves 0, 1, 2, 3
#pragma unroll
            for (int w = 0; w < 3; ++w) v += part[(w * NACC + q * CP + p) * 16 + slot];
            v += W[B.t0off + (int64_t)nn * B.M + m];
            Y[yv.off + pl * yv.poff + (int64_t)jn * yv.ld + m] = v;
        }
}

__global__ __launch_bounds__(kK2Threads, 2) void stage2k(const KS2Block* __restrict__ blks,
                                                         const int64_t* __restrict__ ctab,
                                                         const KTile* __restrict__ tiles,
                                                         const ProbPtrs* __restrict__ probs,
                                                         ProbPtrs single) {
    __shared__ double part[3 * 64 * 16];
    const KTile tl = tiles[blockIdx.x];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const KS2Block B = blks[tl.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    switch (tl.shape) {
#define DMRG_K2(Q, P) \
    case 4 * Q + P: s2_tile<Q, P>(tl, B, ctab, P_, part); break;
        DMRG_K2(3, 3) DMRG_K2(3, 2) DMRG_K2(3, 1) DMRG_K2(3, 0)
        DMRG_K2(2, 3) DMRG_K2(2, 2) DMRG_K2(2, 1) DMRG_K2(2, 0)
        DMRG_K2(1, 3) DMRG_K2(1, 2) DMRG_K2(1, 1) DMRG_K2(1, 0)
        DMRG_K2(0, 3) DMRG_K2(0, 2) DMRG_K2(0, 1) DMRG_K2(0, 0)
#undef DMRG_K2
        default: break;
    }
}

}  // namespace

// Stage 1 of the K-split family: the pre-pack of the input vector, then the tiles.
hipError_t launch_stage1_k(const KXBlock* xblk, const KPItem* pitems, int npitems,
                           const KS1Block* s1, const KEdgeOut* eout, const KTile* t1, int nt1,
                           const ProbPtrs* probs, ProbPtrs single, hipStream_t s) {
    if (npitems > 0)
        hipLaunchKernelGGL(k_prepack, dim3(npitems), dim3(64), 0, s, xblk, pitems, probs, single);
    if (nt1 > 0) hipLaunchKernelGGL(stage1k, dim3(nt1), dim3(64), 0, s, s1, eout, t1, probs, single);
    return hipGetLastError();
}

hipError_t launch_stage2_k(const KS2Block* s2, const int64_t* ctab, const KTile* t2, int nt2,
                           const ProbPtrs* probs, ProbPtrs single, hipStream_t s) {
    if (nt2 > 0)
        hipLaunchKernelGGL(stage2k, dim3(nt2), dim3(kK2Threads), 0, s, s2, ctab, t2, probs, single);
    return hipGetLastError();
}

}  // namespace dmrg
