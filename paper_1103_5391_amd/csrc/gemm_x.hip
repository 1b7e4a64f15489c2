// LDS-staged block products of H_sb.psi on gfx950 (FP64): the two stages of gemm.hip with both
// operands of every K chunk loaded once per work group and shared through LDS by its four
// wavefronts, multiplied with v_mfma_f64_4x4x4_4b_f64.
//
//   stage 1  T_b  = X_b R_b          64 x 64 tiles (the LDS-tiled family's list); each wave 64 x 16
//                                    (all rows, its own 16 columns); K = e, one group per tile
//   stage 2  Y_b' = T0 + Acat Bcat   64 x 32 tiles, waves 2 x 2 of 32 x 16; tiles with long K
//                                    run as two slices that add into a zeroed output
//
// Why this MFMA: on this part v_mfma_f64_16x16x4f64 sustains about 44 TFLOP/s (about 105
// clocks per instruction per SIMD), while v_mfma_f64_4x4x4_4b_f64 sustains about 69 TFLOP/s
// (measured with register operands and several independent accumulators per SIMD).  The 4x4x4
// form needs more operand registers per flop, so the operands come from LDS: a work group's
// tile is four waves' worth, and per 16-deep chunk the work group loads 16 KB (stage 1) or 12 KB
// (stage 2) with 16-byte loads.
//
// The 4x4x4 (four blocks) instruction: lane l = 16 k + 4 b + x supplies A(row x, k) and
// B(k, column x) of block b, and holds D(row t, column j) of block b in lane 16 t + 4 b + j.
// Here the four blocks are the four 4-row groups of one 16-row strip sharing one 4-column piece
// of B, so the A register of a strip is exactly the 16x16x4 fragment (lane 16 g + r: row r, the
// four k = 4 g + step of the chunk, one per instruction step) and the B register of a 4-column
// piece cb reads the 16x16x4 fragment of its panel at lane 16 g + 4 cb + x (each value used by
// the four blocks).  Every step takes k = 4 g + step from lane group g: a fixed permutation of
// the chunk's K on both operands.  The accumulator of (strip s, piece cb) holds rows
// 16 s + 4 b + t (t = l / 16, b = (l / 4) mod 4) of columns 4 cb + (l mod 4): 16 consecutive
// rows of four columns, stored directly (128-byte runs).
//
// LDS layout: per buffer, every 16-row (column) panel of an operand holds its fragments for one
// chunk as two 16-byte halves per lane in separate arrays.  A panels are in lane order (a wave
// reads 1 KB of consecutive bytes); B panels are rotated, lane 16 g + r at 16 g + ((r + 4 g) mod
// 16), so that the sixteen distinct lanes a B-piece read touches fall in distinct banks.
//
// Pipeline: two LDS buffers; iteration c requests chunk c + 1 into registers, multiplies chunk
// c from LDS, then writes chunk c + 1 into the other buffer, one barrier per chunk.
//
// Measured: the family is bound by LDS traffic (about 60 bytes per clock per compute unit for
// 16-byte accesses), and the B pieces of the 4x4x4 form cost a full 16-byte read per lane for 16
// distinct values.  On the half-filled 2 x 16 ladder at m = 1000 the register-tiled kernels are
// faster; on the 2 x 32 ladder at m = 2000 the stage-2 kernel here is.
//
// Split K: two slices of one tile add their products (the first with T0) into an output region
// that extra work groups of the stage-1 launch zeroed; two additions onto zero give the same
// value in either order, so results do not depend on which slice lands first.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mfma.hpp"

namespace dmrg {

namespace {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));   // 16 bytes
typedef double dd2 __attribute__((ext_vector_type(2)));

constexpr int kXT = 256;   // threads of a work group (four wavefronts)

// B panels: half h of rotated lane pos at B[panel][h * kBHalf + pos]; the second half starts
// two bank quads (32 bytes) further, so that the stage-2 loader's 16-lane passes (eight lanes
// per column: four lane groups x two halves) write sixteen distinct bank quads.
constexpr int kBHalf = 64 + 2;

template <int NA, int NB>
struct XStage {
    u4 A[NA][2][64];            // [row panel][half][lane]
    u4 B[NB][2 * kBHalf];       // [column panel][half * kBHalf + rotated lane]
};

// Position of lane 16 g + r of a B panel (rotation by 4 g).
__device__ __forceinline__ int bpos(int lane) {
    const int g = lane >> 4;
    return (g << 4) | (((lane & 15) + 4 * g) & 15);
}

__device__ __forceinline__ d4 frag_of(const u4& lo, const u4& hi) {
    union {
        u4 h[2];
        d4 f;
    } u;
    u.h[0] = lo;
    u.h[1] = hi;
    return u.f;
}

__device__ __forceinline__ u4 pack2(double a, double b) {
    union {
        dd2 d;
        u4 h;
    } u;
    u.d = (dd2){a, b};
    return u.h;
}

// acc[s][cb] += strip s of A x piece cb of B over the chunk's four steps; FULL: every strip
// and piece, else only the valid strips (vs) and pieces (vc), wave-uniform.
template <bool FULL, int NS, int NC>
__device__ __forceinline__ void mma4(double (&acc)[NS][NC], const d4 (&fa)[NS], const d4 (&fb)[NC],
                                     int vs, int vc) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (FULL || (s < vs && c < vc))
                    acc[s][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[s][t], fb[c][t], acc[s][c], 0, 0, 0);
}

// Valid 16-row strips (0..NS) of a range of NS strips starting at `start` of an extent; valid
// 4-column pieces (0..NC) likewise.
template <int NS>
__device__ __forceinline__ int valid_strips(int start, int extent) {
    const int left = extent - start;
    return left <= 0 ? 0 : (left >= 16 * NS ? NS : (left + 15) / 16);
}
template <int NC>
__device__ __forceinline__ int valid_pieces(int start, int extent) {
    const int left = extent - start;
    return left <= 0 ? 0 : (left >= 4 * NC ? NC : (left + 3) / 4);
}

// Runs the chunks [c0, c1) of a work group through two LDS buffers with the loads two chunks
// ahead: register set r1 holds the chunk after the one being multiplied (in flight), r0 takes the
// one after that.  Every load of the main loop is unconditional (the last two chunks are peeled),
// so the compiler's wait before each store counts exactly the newer loads still allowed in flight;
// scheduling barriers keep the loads ahead of the products and each store (with its wait) after
// them.
//   load(c, regs)        issue the global loads of chunk c into a register set
//   store(buf, regs)     write a register set into LDS buffer buf
//   compute(buf)         multiply the chunk in LDS buffer buf
// Runs the chunks [c0, c1) of a work group through two LDS buffers: iteration c requests chunk
// c + 1 into registers, multiplies chunk c from LDS, then writes chunk c + 1 into the other
// buffer, one barrier per chunk.  (A second register set, loads two chunks ahead, measured slower
// on this part: the kernels are bound by LDS traffic, and the extra registers cost occupancy.)
//   load(c, regs)        issue the global loads of chunk c into the register set
//   store(buf, regs)     write the register set into LDS buffer buf
//   compute(buf)         multiply the chunk in LDS buffer buf
template <class R, class Load, class Store, class Compute>
__device__ __forceinline__ void pipeline1(int c0, int c1, Load&& load, Store&& store, Compute&& compute) {
    R r;
    const int last = c1 - 1;
    load(c0, r);
    store(0, r);
    __syncthreads();
    for (int c = c0; c <= last; ++c) {
        const int buf = (c - c0) & 1;
        load(min(c + 1, last), r);   // the next chunk in flight (the last one repeated)
        __builtin_amdgcn_sched_barrier(0);
        compute(buf);
        __builtin_amdgcn_sched_barrier(0);
        store(buf ^ 1, r);           // the other buffer: every wave has left it (barrier)
        __syncthreads();
    }
}

}  // namespace

// ---------------------------------------------------------------------------------------
// stage 1: blocks [0, ntiles) take 64 x 64 tiles, blocks [ntiles, ntiles + nzero) zero one
// 64 x 32 output region of a split stage-2 tile each
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kXT, 2) void stage1x(const S1Block* __restrict__ blks,
                                                  const LItem1* __restrict__ tiles, int ntiles,
                                                  const S2Block* __restrict__ blks2,
                                                  const XZero* __restrict__ zs, int nzero,
                                                  const ProbPtrs* __restrict__ probs,
                                                  ProbPtrs single) {
    const int tid = threadIdx.x;
    if ((int)blockIdx.x >= ntiles) {
        const int zi = (int)blockIdx.x - ntiles;
        if (zi >= nzero) return;
        const XZero z = zs[zi];
        const S2Block B = blks2[z.blk];
        const ProbPtrs P_ = probs ? probs[B.prob] : single;
        if (P_.skip && *P_.skip) return;
        const int m = z.m0 + (tid & 63);
        if (m < B.M) {
            double* __restrict__ Y = P_.y;
            for (int j = tid >> 6; j < kXTile2N; j += kXT / 64) {
                const int n = z.n0 + j;
                if (n < B.N) {
                    const int pl = n >= B.Y.split;
                    Y[B.Y.off + pl * B.Y.poff + (int64_t)(n - pl * B.Y.split) * B.Y.ld + m] = 0.0;
                }
            }
        }
        return;
    }
    const LItem1 tl = tiles[blockIdx.x];
    if (tl.blk < 0) return;   // padding of the XCD-ordered list
    const S1Block B = blks[tl.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    __shared__ XStage<4, 4> sm[2];
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // column panel of the wave
    const int K = B.K, nch = (K + PF64::CK - 1) / PF64::CK;
    // X loader: row lrow of the tile, k = 4 kg + j of each chunk -> lane (kg, lrow mod 16) of
    // row panel lrow / 16
    const int lrow = tid & 63, kg = tid >> 6;
    int64_t arow;
    {
        const int m = min(tl.m0 + lrow, B.M - 1);    // rows beyond M: any valid row, not stored
        const int pl = m >= B.X.split;
        arow = B.X.off + pl * B.X.poff + (m - pl * B.X.split);
    }
    const double* __restrict__ X = P_.x;
    const int64_t ldx = B.X.ld;
    const int apanel = lrow >> 4, alane = kg * 16 + (lrow & 15);
    // R loader: lane `lane` of column panel tid / 64 (packed: [panel][chunk][64 lanes][4])
    const int rpanel = tid >> 6, rpos = bpos(lane);
    const double* rp = static_cast<const double*>(P_.Rops) + B.Roff +
                       ((int64_t)(tl.n0 / kPanel + rpanel) * nch * 64 + lane) * 4;
    struct Regs {
        double xa[4];
        u4 rlo, rhi;
    };
    auto load = [&](int c, Regs& r) {
        const int kb = c * PF64::CK + 4 * kg;
#pragma unroll
        for (int j = 0; j < 4; ++j) r.xa[j] = ldg(X, arow + (int64_t)min(kb + j, K - 1) * ldx);
        const double* q = rp + (int64_t)c * 256;
        r.rlo = ldgv<u4>(q);
        r.rhi = ldgv<u4>(q + 2);
    };
    auto store = [&](int buf, const Regs& r) {
        sm[buf].A[apanel][0][alane] = pack2(r.xa[0], r.xa[1]);
        sm[buf].A[apanel][1][alane] = pack2(r.xa[2], r.xa[3]);
        sm[buf].B[rpanel][rpos] = r.rlo;
        sm[buf].B[rpanel][kBHalf + rpos] = r.rhi;
    };
    // reader of piece cb of the wave's panel: lane 16 g + 4 cb + x of the 16x16x4 fragment
    int bread[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) bread[cb] = bpos(((lane >> 4) << 4) | (4 * cb) | (lane & 3));
    const int vs = valid_strips<4>(tl.m0, B.M), vc = valid_pieces<4>(tl.n0 + 16 * wave, B.N);
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    // the chunk loop, once for whole tiles and once for ragged ones (vs, vc are loop-invariant)
    auto run = [&](auto full) {
        pipeline1<Regs>(0, nch, load, store, [&](int buf) {
            if (vc > 0) {
                d4 fa[4], fb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    fa[i] = frag_of(sm[buf].A[i][0][lane], sm[buf].A[i][1][lane]);
                    fb[i] = frag_of(sm[buf].B[wave][bread[i]], sm[buf].B[wave][kBHalf + bread[i]]);
                }
                mma4<decltype(full)::value, 4, 4>(acc, fa, fb, vs, vc);
            }
        });
    };
    if (vs == 4 && vc == 4)
        run(std::true_type{});
    else
        run(std::false_type{});
    double* __restrict__ T = static_cast<double*>(P_.T);
    const View tv = B.T;
    const int t = lane >> 4, b = (lane >> 2) & 3, j = lane & 3;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int m = tl.m0 + 16 * s + 4 * b + t;
        if (m >= B.M) continue;
        const int pl = m >= tv.split;
        const int64_t rbase = tv.off + pl * tv.poff + (m - pl * tv.split);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int n = tl.n0 + 16 * wave + 4 * cb + j;
            if (n < B.N) T[rbase + (int64_t)n * tv.ld] = acc[s][cb];
        }
    }
}

// ---------------------------------------------------------------------------------------
// stage 2: one 64 x 32 output tile (or one K slice of it) per work group
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kXT, 2) void stage2x(const S2Block* __restrict__ blks,
                                                  const XChunk* __restrict__ ctab,
                                                  const XItem2* __restrict__ items,
                                                  const ProbPtrs* __restrict__ probs,
                                                  ProbPtrs single) {
    const XItem2 it = items[blockIdx.x];
    if (it.blk < 0) return;   // padding of the XCD-ordered list
    const S2Block B = blks[it.blk];
    const ProbPtrs P_ = probs ? probs[B.prob] : single;
    if (P_.skip && *P_.skip) return;
    __shared__ XStage<4, 2> sm[2];
    __shared__ int64_t s_off[kXMaxItemChunks], s_poff[kXMaxItemChunks];
    __shared__ int32_t s_ld[kXMaxItemChunks];
    const int tid = threadIdx.x, lane = tid & 63;
    // the item's chunk sources (at most kXMaxItemChunks, planner's guarantee) into LDS first
    for (int t = tid; t < it.kc1 - it.kc0; t += kXT) {
        const XChunk e = ctab[it.ctab0 + it.kc0 + t];
        s_off[t] = e.off;
        s_poff[t] = e.poff;
        s_ld[t] = e.ld;
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 1, wn = wave >> 1;
    const int split = B.Y.split;   // columns per plane of the output and of every source
    // A loader: lane `lane` of row panel tid / 64 (packed left factors, 64-row tiles)
    const int apanel = tid >> 6;
    const double* ap = static_cast<const double*>(P_.Lops) + B.Aoff +
                       ((int64_t)(it.m0 / kPanel + apanel) * B.nch * 64 + lane) * 4;
    // B loader: column j of the tile, k = 2 q, 2 q + 1 of the chunk -> half q mod 2 of lane
    // (q / 2, j mod 16) of column panel j / 16 (eight consecutive lanes read one column's 128
    // bytes)
    const int jc = tid >> 3, q = tid & 7, kq = 2 * q;
    const int n = min(it.n0 + jc, B.N - 1);    // columns beyond N: any valid column, not stored
    const int pl = n >= split, col = n - pl * split;
    const int bpanel = jc >> 4, bslot = (q & 1) * kBHalf + bpos((q >> 1) * 16 + (jc & 15));
    const double* __restrict__ xin = P_.x;
    const double* __restrict__ tws = static_cast<const double*>(P_.T);
    const int K0 = B.M;   // segment 0 (the diagonal H_S term) reads the block from x: K0 rows
    const int nch0 = (K0 + PF64::CK - 1) / PF64::CK;
    struct Regs {
        u4 alo, ahi, bv;
    };
    auto load = [&](int c, Regs& r) {
        const double* qa = ap + (int64_t)c * 256;
        r.alo = ldgv<u4>(qa);
        r.ahi = ldgv<u4>(qa + 2);
        const int t = c - it.kc0;
        const int k = c * PF64::CK + kq;
        const int64_t base = s_off[t] + pl * s_poff[t] + (int64_t)col * s_ld[t];
        if (c < nch0) {     // input vector: rows beyond K0 clamped (their factors are zero)
            r.bv = pack2(ldg(xin, base + min(k, K0 - 1)), ldg(xin, base + min(k + 1, K0 - 1)));
        } else {            // workspace: zero-padded whole chunks, 16-byte aligned pairs
            r.bv = ldgv<u4>(tws + base + k);
        }
    };
    auto store = [&](int buf, const Regs& r) {
        sm[buf].A[apanel][0][lane] = r.alo;
        sm[buf].A[apanel][1][lane] = r.ahi;
        sm[buf].B[bpanel][bslot] = r.bv;
    };
    int bread[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) bread[cb] = bpos(((lane >> 4) << 4) | (4 * cb) | (lane & 3));
    const int vs = valid_strips<2>(it.m0 + 32 * wm, B.M);
    const int vc = valid_pieces<4>(it.n0 + 16 * wn, B.N);
    double acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    auto run = [&](auto full) {
        pipeline1<Regs>(it.kc0, it.kc1, load, store, [&](int buf) {
            if (vs > 0 && vc > 0) {
                d4 fa[2], fb[4];
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    fa[i] = frag_of(sm[buf].A[2 * wm + i][0][lane], sm[buf].A[2 * wm + i][1][lane]);
#pragma unroll
                for (int cb = 0; cb < 4; ++cb)
                    fb[cb] = frag_of(sm[buf].B[wn][bread[cb]], sm[buf].B[wn][kBHalf + bread[cb]]);
                mma4<decltype(full)::value, 2, 4>(acc, fa, fb, vs, vc);
            }
        });
    };
    if (vs == 2 && vc == 4)
        run(std::true_type{});
    else
        run(std::false_type{});
    if (vs == 0 || vc == 0) return;
    double* __restrict__ Y = P_.y;
    const View t0 = B.T0, yv = B.Y;
    const int t = lane >> 4, b = (lane >> 2) & 3, j = lane & 3;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int nn = it.n0 + 16 * wn + 4 * cb + j;
        if (nn >= B.N) continue;
        const int p2 = nn >= split, c2 = nn - p2 * split;
        const int64_t ybase = yv.off + p2 * yv.poff + (int64_t)c2 * yv.ld;
        const int64_t tbase = t0.off + p2 * t0.poff + (int64_t)c2 * t0.ld;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int m = it.m0 + 32 * wm + 16 * s + 4 * b + t;
            if (m >= B.M) continue;
            double val = acc[s][cb];
            if (it.mode != 2) val = tws[tbase + m] + val;
            if (it.mode == 0)
                Y[ybase + m] = val;
            else
                unsafeAtomicAdd(Y + ybase + m, val);
        }
    }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
hipError_t launch_stage1_x(const S1Block* blks, const LItem1* tiles, int ntiles,
                           const S2Block* blks2, const XZero* zs, int nzero,
                           const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    if (ntiles + nzero == 0) return hipSuccess;
    hipLaunchKernelGGL(stage1x, dim3(ntiles + nzero), dim3(kXT), 0, st, blks, tiles, ntiles, blks2,
                       zs, nzero, probs, single);
    return hipGetLastError();
}

hipError_t launch_stage2_x(const S2Block* blks, const XChunk* ctab, const XItem2* items, int nitems,
                           const ProbPtrs* probs, ProbPtrs single, hipStream_t st) {
    if (nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(stage2x, dim3(nitems), dim3(kXT), 0, st, blks, ctab, items, probs, single);
    return hipGetLastError();
}

}  // namespace dmrg
