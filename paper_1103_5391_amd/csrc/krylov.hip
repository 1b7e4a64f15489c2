// Lanczos vector kernels, tridiagonal exponential and Krylov combination (FP64, gfx950).
//
// Sec. II.A: the Lanczos recursion is started from phi itself, H ~ V^T T V, and
//   phi(t) ~ beta0 V^T S exp(-i D t) S^T e_1,     T = S D S^T.
// Storage: slot j of the basis buffer holds u_j = beta_j v_j (the vector before
// normalisation) and the state keeps scale[j] = 1/beta_j, so no separate normalisation pass
// is needed; every consumer multiplies by scale[j] on load.
//
// Orthogonalisation: full reorthogonalisation by two classical Gram-Schmidt sweeps against
// the whole basis, with the second sweep of each new vector delayed into the next iteration so
// that one iteration is one reduction pass, a small totals kernel and one update pass.  Slot j
// holds u1, the new vector after its first sweep, when iteration j starts; the block products
// are applied to that slot as it is (w_raw = H u1).  Then
//   reduce    a = V^H u1, b = V^H w_raw (slots c < j), c = u1^H w_raw, d = ||u1||^2,
//             e = ||w_raw||^2                                             (one pass)
//   algebra   (O(j) work, repeated by every block of the update pass)
//             second sweep of u1: u = u1 - V a, beta_j^2 = d - |a|^2, v_j = u / beta_j;
//             H u = w_raw - H V a, where H V a = V T a up to second order in the loss of
//             orthogonality (T: the Lanczos matrix so far), so w = H v_j is known in the basis:
//             h_c = v_c^H w = (b_c - t_c) / beta_j (c < j), t = T a,
//             h_j = (c - a^H b) / beta_j^2 - t_j / beta_j, alpha_j = Re h_j
//   update    slot j <- u; slot j+1 <- w - sum_c h_c v_c (first sweep of the next vector;
//             it contains the three-term recurrence, whose coefficients are h_j and h_{j-1})
//                                                                          (one pass)
// In exact arithmetic this is the two-sweep recurrence; the dropped terms are products of two
// quantities of the order of the loss of orthogonality.
//
// Every kernel runs over a table of problems (one entry for a single superblock, many for a
// batch): block b of a pass works on problem bmap[b] (problem 0 when there is no map), as block
// b - b0 of that problem's nb blocks; the small kernels run one block (or a few) per problem.
// The three kernels of a Lanczos iteration have a second instance for a lone problem, which
// takes its descriptor by value instead of from the table.
// Grid-wide sums are deterministic: every block writes its partial sums and a later kernel adds
// them in a fixed order (the kernel boundary orders the two; no device-wide fences or atomics:
// on this chip a device-scope release writes back the XCD's L2 and costs more than a launch).
#include <array>
#include <utility>

#include "internal.hpp"

namespace dmrg {

static_assert(kDVals % (kVecThreads / 64) == 0, "k_dsum: whole blocks of values");

namespace {

typedef const double __attribute__((address_space(1)))* gcptr;

typedef double d2v __attribute__((ext_vector_type(2)));
// Elements i, i + 1 (i even, p 16-byte aligned) of the slot starting at p.
__device__ __forceinline__ d2v ld2(const double* p, int64_t i) {
    return *((const d2v __attribute__((address_space(1)))*)(p + i));
}
__device__ __forceinline__ void st2(double* p, int64_t i, d2v v) {
    *((d2v __attribute__((address_space(1)))*)(p + i)) = v;
}

// Load of element i of the basis slot starting at p (global address space: the uniform slot
// base can live in scalar registers, the lane offset in one vector register).
__device__ __forceinline__ double ldv(const double* p, int64_t i) { return ((gcptr)p)[i]; }

// DPP move of a double (both 32-bit halves) with the given data-parallel-primitive control.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_read(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront, returned in every lane: butterflies inside each row of
// 16 lanes with DPP (quad swaps, half-row and row mirrors), then the four row sums read out
// with readlane.  Fixed order, no LDS traffic.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);   // row_half_mirror: lane i <-> 7 - i within each half row
    v += dpp<0x140>(v);   // row_mirror: lane i <-> 15 - i within the row
    return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

// Where block blockIdx.x of a pass works: problem bmap[blockIdx.x / mult] (0 without a map),
// block lb of the nbt = nb * mult blocks that pass gives that problem.
struct Where {
    VecProb p;
    int prob, lb, nbt;
};
__device__ __forceinline__ Where locate(const VecProb* vp, const int* bmap, int mult) {
    Where w;
    w.prob = bmap ? bmap[blockIdx.x / mult] : 0;
    w.p = vp[w.prob];
    w.lb = (int)blockIdx.x - w.p.b0 * mult;
    w.nbt = w.p.nb * mult;
    return w;
}

// The per-iteration passes are instantiated twice: ONE for a lone problem, whose descriptor
// comes by value with the kernel arguments (`one`), so the first data loads wait for no global
// load of a table entry; otherwise the table vp and the block map.  (A run-time choice between
// the two would read the descriptor through a generic pointer.)
template <bool ONE>
__device__ __forceinline__ Where locate1(const VecProb* vp, const int* bmap, const VecProb& one) {
    Where w;
    if constexpr (ONE) {
        w.prob = 0;
        w.p = one;
    } else {
        w.prob = bmap[blockIdx.x];
        w.p = vp[w.prob];
    }
    w.lb = (int)blockIdx.x - w.p.b0;
    w.nbt = w.p.nb;
    return w;
}

// The same for the reduction pass, which has its own block decomposition (nbr blocks per problem,
// several elements per thread, so that the per-block sums of its many values are amortised).
template <bool ONE>
__device__ __forceinline__ Where locate_red(const VecProb* vp, const int* bmapr,
                                            const VecProb& one) {
    Where w;
    if constexpr (ONE) {
        w.prob = 0;
        w.p = one;
    } else {
        w.prob = bmapr[blockIdx.x];
        w.p = vp[w.prob];
    }
    w.lb = (int)blockIdx.x - w.p.b0r;
    w.nbt = w.p.nbr;
    return w;
}

// Block-level sums of NV per-thread values; writes the block partials value-major,
// part[v * kVecMaxBlocks + lb], so that the finalise block reads each value's rows contiguously.
template <int NV>
__device__ __forceinline__ void block_partials(const double (&vals)[NV], double* part, int lb) {
    __shared__ double red[NV][kVecThreads / 64];
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][wave] = wave_sum(vals[v]);   // every lane holds the sum
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kVecThreads / 64; ++w) s += red[v][w];
        part[(int64_t)v * kVecMaxBlocks + lb] = s;
    }
}

// As block_partials for NV values, then zeros for values NV .. ROW-1.
template <int NV, int ROW>
__device__ __forceinline__ void block_partials_row(const double (&vals)[NV > 0 ? NV : 1],
                                                   double* part, int lb) {
    __shared__ double red[NV > 0 ? NV : 1][kVecThreads / 64];
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][wave] = wave_sum(vals[v]);   // every lane holds the sum
    __syncthreads();
    for (int v = threadIdx.x; v < ROW; v += blockDim.x) {
        double s = 0.0;
        if (v < NV) {
#pragma unroll
            for (int w = 0; w < kVecThreads / 64; ++w) s += red[v][w];
        }
        part[(int64_t)v * kVecMaxBlocks + lb] = s;
    }
}

// Exchange partner for the reduce-scatter step on lane bit B: lane ^ B for the bits that cross
// rows of 16 (through the LDS permute network), otherwise a DPP move within the row whose
// partner differs in bit B (and possibly lower bits, which are not yet reduced).
template <int B>
__device__ __forceinline__ double partner(double v) {
    if constexpr (B >= 16) return __shfl_xor(v, B, 64);
    else if constexpr (B == 8) return dpp<0x140>(v);   // row_mirror: lane i <-> 15 - i
    else if constexpr (B == 4) return dpp<0x141>(v);   // row_half_mirror: i <-> 7 - i
    else if constexpr (B == 2) return dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    else return dpp<0xB1>(v);                          // quad_perm [1,0,3,2]
}

// Reduce-scatter of P (a power of two, <= 64) per-lane values over the wavefront by recursive
// halving: at the step on lane bit B a lane keeps the half of its remaining values selected by
// that bit and adds its partner's copy of the same half; after log2 P steps each lane holds one
// value, the wavefront sum of value index lane >> (6 - log2 P), and the remaining lane bits are
// summed by plain butterflies.  P - 1 + 6 - log2 P exchanges instead of 6 P for P wave sums.
template <int P, int B = 32>
__device__ __forceinline__ void halve(double (&v)[P], int lane) {
    if constexpr (P > 1) {
        constexpr int H = P / 2;
        const bool upper = lane & B;
        double keep[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double give = upper ? v[i] : v[i + H];
            const double mine = upper ? v[i + H] : v[i];
            keep[i] = mine + partner<B>(give);
        }
        double (&w)[H] = *reinterpret_cast<double(*)[H]>(v);
#pragma unroll
        for (int i = 0; i < H; ++i) w[i] = keep[i];
        halve<H, B / 2>(w, lane);
    } else if constexpr (B >= 1) {
        v[0] += partner<B>(v[0]);
        halve<1, B / 2>(v, lane);
    }
}

// Block-level sums of NV <= 64 per-thread values by wavefront reduce-scatter, written as a row
// of ROW values (zeros past NV), value-major: part[v * kVecMaxBlocks + lb].
template <int NV, int ROW>
__device__ __forceinline__ void block_partials_scatter(const double (&vals)[NV > 0 ? NV : 1],
                                                       double* part, int lb) {
    static_assert(NV <= 64 && ROW <= 64, "one value per lane");
    constexpr int P = NV <= 1 ? 1 : NV <= 2 ? 2 : NV <= 4 ? 4 : NV <= 8 ? 8 : NV <= 16 ? 16
                                                         : NV <= 32 ? 32 : 64;
    constexpr int SHIFT = P == 1 ? 6 : P == 2 ? 5 : P == 4 ? 4 : P == 8 ? 3 : P == 16 ? 2
                                                   : P == 32 ? 1 : 0;
    __shared__ double red[kVecThreads / 64][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[P];
#pragma unroll
    for (int i = 0; i < P; ++i) v[i] = i < NV ? vals[i] : 0.0;
    halve<P>(v, lane);
    if ((lane & ((1 << SHIFT) - 1)) == 0) red[wave][lane >> SHIFT] = v[0];
    __syncthreads();
    for (int i = threadIdx.x; i < ROW; i += blockDim.x) {
        double s = 0.0;
        if (i < NV) {
#pragma unroll
            for (int w = 0; w < kVecThreads / 64; ++w) s += red[w][i];
        }
        part[(int64_t)i * kVecMaxBlocks + lb] = s;
    }
}

// Finalise kernels run one block of FT threads per problem: totals[v] = sum_b part[v][b] for
// v < NV in a fixed order (thread t adds rows t, t + FT, ... in turn, then the block reduction
// of block_partials; nb <= kVecMaxBlocks, value-major layout as written by block_partials).
template <int NV, int FT = kVecThreads>
__device__ void final_sums(const double* part, int nb, double* totals_lds) {
    __shared__ double red[NV][FT / 64];
    const int wave = threadIdx.x >> 6;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    // global-address-space loads: all NV of a row group are requested before the first use
    const gcptr gp = (gcptr)part;
#pragma unroll 1
    for (int q = 0; q < kVecMaxBlocks / FT; ++q) {
        const int b0 = q * FT + threadIdx.x;
        const int b = b0 < nb ? b0 : nb - 1;
        const double keep = b0 < nb ? 1.0 : 0.0;
        double x[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = gp[(int64_t)v * kVecMaxBlocks + b];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += x[v] * keep;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][wave] = wave_sum(acc[v]);   // every lane holds the sum
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += FT) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < FT / 64; ++w) t += red[v][w];
        totals_lds[v] = t;
    }
    __syncthreads();
}

// Starts a Krylov step from ||x||^2: beta0, scale0, per-step flags.
__device__ void begin_step(KState* st, double norm2, int kdim) {
    double b0 = sqrt(norm2);
    if (!isfinite(b0)) {          // NaN or infinity in the vector: flagged, run as zero
        st->nonfinite = 1;
        b0 = 0.0;
    }
    st->beta[0] = b0;
    st->kdim = kdim;
    if (b0 > 0.0) {
        st->scale[0] = 1.0 / b0;
        st->keff = kdim;
        st->broken = 0;
    } else {
        st->scale[0] = 0.0;
        st->keff = 0;
        st->broken = 1;
    }
}

}  // namespace

// ---------------------------------------------------------------------------------------
// start: slot 0 <- x, partial ||x||^2.  x is x1 (one problem) or xt[problem] (a batch).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_start(const VecProb* vp, const int* bmap,
                                                       const double* x1,
                                                       const double* const* xt) {
    const Where W = locate(vp, bmap, 1);
    const double* __restrict__ x = xt ? xt[W.prob] : x1;
    double* __restrict__ u0 = W.p.V;
    const int64_t n = W.p.n;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)W.nbt * blockDim.x;
    for (int64_t i = (int64_t)W.lb * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double re = x[i], im = x[n + i];
        u0[i] = re;
        u0[n + i] = im;
        acc[0] += re * re + im * im;
    }
    block_partials<1>(acc, W.p.part, W.lb);
}

__global__ __launch_bounds__(kVecThreads) void k_fin_start(const VecProb* vp, int kdim, int first) {
    const VecProb P = vp[blockIdx.x];
    KState* st = P.st;
    __shared__ double tot[1];
    final_sums<1>(P.part, P.nb, tot);
    if (threadIdx.x == 0) {
        if (first) st->nonfinite = 0;
        begin_step(st, tot[0], kdim);
        st->err_est = 0.0;
        st->exp_fail = 0;
        if (first) {
            st->keff_min = kMaxKrylov + 1;
            st->any_break = 0;
            st->beta0_first = st->beta[0];
        }
    }
}

// ---------------------------------------------------------------------------------------
// Lanczos iteration j: reduction pass.  Launch q covers slots c0 .. c0+NC-1 (NC <= kDSlots);
// the first launch also accumulates u1^H w_raw, ||u1||^2 and ||w_raw||^2.  Partial rows of
// launch q: kDVals values (a_c, b_c per slot, then c, d, e), unused values zero.
// ---------------------------------------------------------------------------------------
template <int NC, bool FIRST, bool ONE>
__global__ __launch_bounds__(kVecThreads) void k_dreduce(const VecProb* vp, const int* bmap, int j,
                                                         int c0, int q, VecProb one) {
    constexpr int NV = 4 * NC + (FIRST ? 4 : 0);
    const Where W = locate_red<ONE>(vp, bmap, one);
    // No breakdown test: the pass writes only its partial rows, which the totals kernel ignores
    // after a breakdown (the slots stay allocated, so every load is in bounds); a test here
    // would put the flag's load before the first data load.
    const double* __restrict__ V0 = W.p.V + (int64_t)c0 * W.p.vstride;
    const double* __restrict__ u1 = W.p.V + (int64_t)j * W.p.vstride;
    const double* __restrict__ w = W.p.w;
    const int64_t n = W.p.n, vstride = W.p.vstride;
    double acc[NV > 0 ? NV : 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    const int64_t stride = (int64_t)W.nbt * blockDim.x;
    if ((n & 1) == 0) {
        for (int64_t i = 2 * ((int64_t)W.lb * blockDim.x + threadIdx.x); i < n; i += 2 * stride) {
            d2v vr[NC > 0 ? NC : 1], vi[NC > 0 ? NC : 1];
            const d2v ur = ld2(u1, i), ui = ld2(u1, n + i), wr = ld2(w, i), wi = ld2(w, n + i);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double* v = V0 + (int64_t)c * vstride;
                vr[c] = ld2(v, i);
                vi[c] = ld2(v, n + i);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    acc[4 * c] += vr[c][h] * ur[h] + vi[c][h] * ui[h];
                    acc[4 * c + 1] += vr[c][h] * ui[h] - vi[c][h] * ur[h];
                    acc[4 * c + 2] += vr[c][h] * wr[h] + vi[c][h] * wi[h];
                    acc[4 * c + 3] += vr[c][h] * wi[h] - vi[c][h] * wr[h];
                }
                if (FIRST) {
                    acc[4 * NC] += ur[h] * wr[h] + ui[h] * wi[h];
                    acc[4 * NC + 1] += ur[h] * wi[h] - ui[h] * wr[h];
                    acc[4 * NC + 2] += ur[h] * ur[h] + ui[h] * ui[h];
                    acc[4 * NC + 3] += wr[h] * wr[h] + wi[h] * wi[h];
                }
            }
        }
    } else
    for (int64_t i = (int64_t)W.lb * blockDim.x + threadIdx.x; i < n; i += stride) {
        // every load of the element first, then the arithmetic (one memory round trip)
        double vr[NC > 0 ? NC : 1], vi[NC > 0 ? NC : 1];
        const double ur = ldv(u1, i), ui = ldv(u1, n + i), wr = ldv(w, i), wi = ldv(w, n + i);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* v = V0 + (int64_t)c * vstride;
            vr[c] = ldv(v, i);
            vi[c] = ldv(v, n + i);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            acc[4 * c] += vr[c] * ur + vi[c] * ui;
            acc[4 * c + 1] += vr[c] * ui - vi[c] * ur;
            acc[4 * c + 2] += vr[c] * wr + vi[c] * wi;
            acc[4 * c + 3] += vr[c] * wi - vi[c] * wr;
        }
        if (FIRST) {
            acc[4 * NC] += ur * wr + ui * wi;
            acc[4 * NC + 1] += ur * wi - ui * wr;
            acc[4 * NC + 2] += ur * ur + ui * ui;
            acc[4 * NC + 3] += wr * wr + wi * wi;
        }
    }
    block_partials_scatter<NV, kDVals>(acc, W.p.part + (int64_t)q * kVecMaxBlocks * kDVals, W.lb);
}

// Lanczos iteration j: totals of the reduction launches.  Wave w of block (x, problem) sums
// value v = 4 x + w of the nq * kDVals values over the nbr partial rows (fixed order: lane l
// adds rows l, l + 64, ... in turn, then the wavefront sum) into the state; many blocks, so the
// partial rows are read in parallel across the chip rather than through one compute unit.
template <bool ONE>
__global__ __launch_bounds__(kVecThreads) void k_dsum(const VecProb* vp, VecProb one) {
    const VecProb P = ONE ? one : vp[blockIdx.y];
    KState* st = P.st;
    const int broken = ((const int __attribute__((address_space(1)))*)&st->broken)[0];
    const int lane = threadIdx.x & 63;
    const int v = blockIdx.x * (kVecThreads / 64) + (threadIdx.x >> 6);
    const gcptr row = (gcptr)(P.part + (int64_t)v * kVecMaxBlocks);
    const int nbr = P.nbr;
    double x[kVecMaxBlocks / 64];
#pragma unroll
    for (int k = 0; k < kVecMaxBlocks / 64; ++k) {
        const int b = lane + 64 * k;
        x[k] = row[b < nbr ? b : nbr - 1] * (b < nbr ? 1.0 : 0.0);
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < kVecMaxBlocks / 64; ++k) acc += x[k];
    acc = wave_sum(acc);
    if (lane == 0 && !broken) st->red[v] = acc;
}

// Lanczos iteration j: the small algebra of the iteration (see the top of this file), run by
// every block of the update pass from the totals of the reduction launches (row layout as
// above; the first launch has nc0 = min(j, kDSlots) slots) and the Lanczos matrix so far, so
// that no one-block launch sits between the reduction and the update.  Every block computes
// the same values in the same order; block 0 of the problem (`writer`) stores alpha_j, beta_j,
// scale_j, the breakdown flag and, on the last iteration, beta_{j+1} from ||w||^2 - |h|^2 for
// the error estimate.  The other blocks read only entries < j of the state, which no block
// writes here.  Result in LDS: co[0][c] = a_c scale_c, co[1][c] = t_c scale_c,
// co[2][c] = h_c scale_c (c < j, zero up to j8), cj = {scale_j, t_j scale_j, h_j scale_j}.
// Returns false (block-uniform) when the basis has broken down.
__device__ __forceinline__ bool iteration_coefficients(KState* st, int j, int kdim, int nc0,
                                                       bool writer, int j8,
                                       int broken, double (&co)[3][2 * kMaxKrylov], double (&cj)[5]) {
    const int tid = threadIdx.x, lane = tid & 63;
    __shared__ double al[kMaxKrylov], be[kMaxKrylov + 1];
    __shared__ double A[2 * kMaxKrylov], Bv[2 * kMaxKrylov], T[2 * kMaxKrylov + 2], sc[kMaxKrylov];
    __shared__ double cde[4], sh[4];
    __shared__ int ok;
    const gcptr red = (gcptr)st->red;
    const double cdev = red[4 * nc0 + (tid & 3)];   // issued with the loads below
    for (int c = tid; c < j; c += blockDim.x) {
        const double s = ((gcptr)st->scale)[c];
        al[c] = ((gcptr)st->alpha)[c];
        be[c] = ((gcptr)st->beta)[c];
        sc[c] = s;
        const int base = (c / kDSlots) * kDVals + 4 * (c % kDSlots);
        A[2 * c] = s * red[base];
        A[2 * c + 1] = s * red[base + 1];
        Bv[2 * c] = s * red[base + 2];
        Bv[2 * c + 1] = s * red[base + 3];
    }
    if (tid < 4) cde[tid] = cdev;
    __syncthreads();
    if (broken) return false;   // an earlier iteration broke down: nothing is written
    if (tid < 64) {
        // wave 0: |a|^2, u^H w_raw = c - a^H b, and the breakdown scale max(1, |alpha_c|, beta_c)
        // over the iterations before j (lane c holds slot c; j <= kMaxKrylov = 64)
        const bool in = lane < j;
        const double ar = in ? A[2 * lane] : 0.0, ai = in ? A[2 * lane + 1] : 0.0;
        const double br = in ? Bv[2 * lane] : 0.0, bi = in ? Bv[2 * lane + 1] : 0.0;
        const double a2 = wave_sum(ar * ar + ai * ai);
        const double abr = wave_sum(ar * br + ai * bi), abi = wave_sum(ar * bi - ai * br);
        double m = in ? fabs(al[lane]) : 0.0;
        if (in && lane >= 1) m = fmax(m, be[lane]);
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        if (lane == 0) {
            const double bscale = fmax(1.0, m);
            // second sweep of u1: beta_j^2 = ||u1||^2 - |a|^2 (beta_0 = ||x|| from the start)
            double bj = ((gcptr)st->beta)[0];
            int good = 1;
            if (j > 0) {
                bj = sqrt(fmax(cde[2] - a2, 0.0));
                if (bj <= 1e-12 * bscale) good = 0;
            }
            if (writer && j > 0) {
                st->beta[j] = bj;
                if (good) {
                    st->scale[j] = 1.0 / bj;
                } else {
                    st->broken = 1;
                    st->keff = j;
                }
            }
            be[j] = bj;
            sh[0] = bj;
            sh[1] = cde[0] - abr;   // u^H w_raw
            sh[2] = cde[1] - abi;
            ok = good;
        }
    }
    __syncthreads();
    if (!ok) return false;
    const double bj = sh[0], ib = 1.0 / bj;
    // t = T a (m = 0 .. j): T[m][m] = alpha_m, T[m][m-1] = beta_m, T[m][m+1] = beta_{m+1}
    for (int m = tid; m <= j; m += blockDim.x) {
        double tr = 0.0, ti = 0.0;
        if (m < j) {
            tr += al[m] * A[2 * m];
            ti += al[m] * A[2 * m + 1];
        }
        if (m >= 1) {
            tr += be[m] * A[2 * (m - 1)];
            ti += be[m] * A[2 * (m - 1) + 1];
        }
        if (m + 1 < j) {
            tr += be[m + 1] * A[2 * (m + 1)];
            ti += be[m + 1] * A[2 * (m + 1) + 1];
        }
        T[2 * m] = tr;
        T[2 * m + 1] = ti;
    }
    __syncthreads();
    for (int c = tid; c < j8; c += blockDim.x) {
        const bool in = c < j;
        const double s = in ? sc[c] : 0.0;
        co[0][2 * c] = in ? A[2 * c] * s : 0.0;
        co[0][2 * c + 1] = in ? A[2 * c + 1] * s : 0.0;
        co[1][2 * c] = in ? T[2 * c] * s : 0.0;
        co[1][2 * c + 1] = in ? T[2 * c + 1] * s : 0.0;
        co[2][2 * c] = in ? (Bv[2 * c] - T[2 * c]) * ib * s : 0.0;
        co[2][2 * c + 1] = in ? (Bv[2 * c + 1] - T[2 * c + 1]) * ib * s : 0.0;
    }
    if (tid < 64) {
        const double ur = sh[1], ui = sh[2];
        const double hr = ur * ib * ib - T[2 * j] * ib, hi = ui * ib * ib - T[2 * j + 1] * ib;
        if (j == kdim - 1) {
            // ||w||^2 = (e - 2 Re(t^H V^H w_raw) + |t|^2) / beta_j^2, V^H w_raw = (b, (u^H w_raw) / beta_j)
            const bool in = lane < j;
            const double tr = in ? T[2 * lane] : 0.0, ti = in ? T[2 * lane + 1] : 0.0;
            const double br = in ? Bv[2 * lane] : 0.0, bi = in ? Bv[2 * lane + 1] : 0.0;
            const double xr = (br - tr) * ib, xi = (bi - ti) * ib;
            const double tw = wave_sum(tr * br + ti * bi) + T[2 * j] * ur * ib + T[2 * j + 1] * ui * ib;
            const double t2 = wave_sum(tr * tr + ti * ti) + T[2 * j] * T[2 * j] + T[2 * j + 1] * T[2 * j + 1];
            const double h2 = wave_sum(xr * xr + xi * xi) + hr * hr + hi * hi;
            const double w2 = (cde[3] - 2.0 * tw + t2) * ib * ib;
            if (writer && lane == 0) {
                st->beta[j + 1] = sqrt(fmax(w2 - h2, 0.0));
                st->keff = kdim;
            }
        }
        if (lane == 0) {
            if (writer) st->alpha[j] = hr;
            cj[0] = ib;
            cj[1] = T[2 * j] * ib;
            cj[2] = T[2 * j + 1] * ib;
            cj[3] = hr * ib;
            cj[4] = hi * ib;
        }
    }
    __syncthreads();
    return true;
}

// Lanczos iteration j: update pass.  slot j <- u = u1 - sum_c a_c v_c; with v_j = u scale_j and
// w = (w_raw - sum_{c<j} t_c v_c - t_j v_j) scale_j: slot j+1 <- w - sum_{c<j} h_c v_c - h_j v_j
// (skipped after the last iteration).
template <bool ONE>
__global__ __launch_bounds__(kVecThreads) void k_dupdate(const VecProb* vp, const int* bmap, int j,
                                                         int kdim, int nc0, VecProb one) {
    const Where W = locate1<ONE>(vp, bmap, one);
    KState* st = W.p.st;
    const int broken = ((const int __attribute__((address_space(1)))*)&st->broken)[0];
    constexpr int G = 8;                       // basis slots loaded per round trip
    const int j8 = (j + G - 1) / G * G;
    __shared__ double co[3][2 * kMaxKrylov];
    __shared__ double cj[5];
    double* __restrict__ uj = W.p.V + (int64_t)j * W.p.vstride;
    double* __restrict__ un = W.p.V + (int64_t)(j + 1) * W.p.vstride;
    const double* __restrict__ V = W.p.V;
    const double* __restrict__ w = W.p.w;
    const int64_t n = W.p.n, vstride = W.p.vstride;
    const int64_t stride = (int64_t)W.nbt * blockDim.x;
    const bool even = (n & 1) == 0;
    // even length: every element pair's loads of the first G basis slots are issued ahead of
    // its arithmetic, for the first pair before the coefficients, so that their latency
    // overlaps the small algebra; the slots are allocated whatever the state, and nothing is
    // stored after a breakdown
    const int64_t i0 = 2 * ((int64_t)W.lb * blockDim.x + threadIdx.x);
    d2v vr[G], vi[G];
    auto head = [&](int64_t i) {
        if (j > 0) {
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const double* v = V + (int64_t)min(k, j - 1) * vstride;
                vr[k] = ld2(v, i);
                vi[k] = ld2(v, n + i);
            }
        }
    };
    if (even && i0 < n) head(i0);
    if (!iteration_coefficients(st, j, kdim, nc0, W.lb == 0, j8, broken, co, cj)) return;
    const bool last = j == kdim - 1;
    const double sj = cj[0], tjr = cj[1], tji = cj[2], hjr = cj[3], hji = cj[4];
    if (even) {
        for (int64_t i = i0; i < n; i += 2 * stride) {
            if (i != i0) head(i);
            const d2v u0r = ld2(uj, i), u0i = ld2(uj, n + i), w0r = ld2(w, i), w0i = ld2(w, n + i);
            d2v ar = 0.0, ai = 0.0, tr = 0.0, ti = 0.0, hr = 0.0, hi = 0.0;
            for (int c0 = 0; c0 < j; c0 += G) {
                if (c0 > 0) {
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const double* v = V + (int64_t)min(c0 + k, j - 1) * vstride;
                        vr[k] = ld2(v, i);
                        vi[k] = ld2(v, n + i);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const int c = c0 + k;
                    ar += co[0][2 * c] * vr[k] - co[0][2 * c + 1] * vi[k];
                    ai += co[0][2 * c] * vi[k] + co[0][2 * c + 1] * vr[k];
                    tr += co[1][2 * c] * vr[k] - co[1][2 * c + 1] * vi[k];
                    ti += co[1][2 * c] * vi[k] + co[1][2 * c + 1] * vr[k];
                    hr += co[2][2 * c] * vr[k] - co[2][2 * c + 1] * vi[k];
                    hi += co[2][2 * c] * vi[k] + co[2][2 * c + 1] * vr[k];
                }
            }
            const d2v ur = u0r - ar, ui = u0i - ai;
            const d2v wr = (w0r - tr - (tjr * ur - tji * ui)) * sj;
            const d2v wi = (w0i - ti - (tjr * ui + tji * ur)) * sj;
            st2(uj, i, ur);
            st2(uj, n + i, ui);
            if (!last) {
                st2(un, i, wr - hr - (hjr * ur - hji * ui));
                st2(un, n + i, wi - hi - (hjr * ui + hji * ur));
            }
        }
        return;
    }
    for (int64_t i = (int64_t)W.lb * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double u0r = ldv(uj, i), u0i = ldv(uj, n + i), w0r = ldv(w, i), w0i = ldv(w, n + i);
        double ar = 0.0, ai = 0.0, tr = 0.0, ti = 0.0, hr = 0.0, hi = 0.0;
        for (int c0 = 0; c0 < j; c0 += G) {
            // G slots per round trip (slots past j - 1 re-read slot j - 1, zero coefficients)
            double vr[G], vi[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const double* v = V + (int64_t)min(c0 + k, j - 1) * vstride;
                vr[k] = ldv(v, i);
                vi[k] = ldv(v, n + i);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int c = c0 + k;
                ar += co[0][2 * c] * vr[k] - co[0][2 * c + 1] * vi[k];
                ai += co[0][2 * c] * vi[k] + co[0][2 * c + 1] * vr[k];
                tr += co[1][2 * c] * vr[k] - co[1][2 * c + 1] * vi[k];
                ti += co[1][2 * c] * vi[k] + co[1][2 * c + 1] * vr[k];
                hr += co[2][2 * c] * vr[k] - co[2][2 * c + 1] * vi[k];
                hi += co[2][2 * c] * vi[k] + co[2][2 * c + 1] * vr[k];
            }
        }
        const double ur = u0r - ar, ui = u0i - ai;
        const double wr = (w0r - tr - (tjr * ur - tji * ui)) * sj;
        const double wi = (w0i - ti - (tjr * ui + tji * ur)) * sj;
        uj[i] = ur;
        uj[n + i] = ui;
        if (!last) {
            un[i] = wr - hr - (hjr * ur - hji * ui);
            un[n + i] = wi - hi - (hjr * ui + hji * ur);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Small exponential: c(t_x) = beta0 exp(-i T t_x) e_1 for the k x k Lanczos matrix T
// (diagonal alpha, off-diagonal beta_1..beta_{k-1}), one wavefront per problem, lane r holding
// component r.  This is the quantity Sec. II.A obtains from T = S D S^T; on the device it is
// evaluated without the eigen-decomposition (a serial QL chase keeps one wavefront busy for
// ~1e5 cycles): T is shifted by the centre sigma of its Gershgorin interval (radius rho bounds
// ||T - sigma||_2), the vector is advanced from one target time to the next in s substeps of
// length h with rho |h| <= 2, each by the Taylor series of exp(-i h (T - sigma)) to order 30
// (remainder below 2^31 / 31! e^2 ~ 2e-24 relative; the largest term is at most 2, so no
// cancellation), and the phase exp(-i sigma t_x) is applied to the output.  Every term costs one
// tridiagonal product: two neighbour exchanges and three multiply-adds per lane.
// Also the error estimate beta_k |c_{k-1}(t_last)|.
// ---------------------------------------------------------------------------------------
namespace {

constexpr int kTaylorOrder = 30;
constexpr double kTaylorRadius = 2.0;

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

}  // namespace

__global__ __launch_bounds__(64) void k_tridiag_expm(const VecProb* vp, double t0, double t1,
                                                     double t2, double t3, int ntimes,
                                                     int* klog, int step) {
    KState* st = vp[blockIdx.x].st;
    const int r = threadIdx.x;
    const int k = st->keff;
    if (klog && r == 0) klog[step] = k > 0 ? k : 0;     // Lanczos vectors of this step
    if (k <= 0) {
        for (int x = 0; x < ntimes; ++x) {
            st->coef[x][2 * r] = 0.0;
            st->coef[x][2 * r + 1] = 0.0;
        }
        if (r == 0) {
            st->err_est = 0.0;
            st->keff_min = 0;
            st->any_break = 1;
        }
        return;
    }
    const bool in = r < k;
    const double a = in ? st->alpha[r] : 0.0;
    const double bl = (in && r >= 1) ? st->beta[r] : 0.0;     // couples r-1 and r
    const double bu = (r + 1 < k) ? st->beta[r + 1] : 0.0;    // couples r and r+1
    const double reach = fabs(bl) + fabs(bu);
    const double hi = wave_max(in ? a + reach : -INFINITY);
    const double lo = -wave_max(in ? reach - a : -INFINITY);
    const double sigma = 0.5 * (hi + lo), rho = 0.5 * (hi - lo);
    const double d = in ? a - sigma : 0.0;
    const double times[kMaxTimes] = {t0, t1, t2, t3};
    double vr = (r == 0) ? st->beta[0] : 0.0, vi = 0.0;
    double tprev = 0.0, lastr = 0.0, lasti = 0.0;
    int bad = 0;
    for (int x = 0; x < ntimes; ++x) {
        const double dt = times[x] - tprev;
        const double need = rho * fabs(dt) / kTaylorRadius;
        const int64_t nsub = dt == 0.0 ? 0 : (need <= 1.0 ? 1 : (int64_t)ceil(need));
        const double h = nsub ? dt / (double)nsub : 0.0;
        for (int64_t sub = 0; sub < nsub; ++sub) {
            // sum_m (-i h (T - sigma))^m v / m!
            double sr = vr, si = vi, tr = vr, ti = vi;
            for (int m = 1; m <= kTaylorOrder; ++m) {
                const double trm = __shfl_up(tr, 1, 64), tim = __shfl_up(ti, 1, 64);
                const double trp = __shfl_down(tr, 1, 64), tip = __shfl_down(ti, 1, 64);
                const double ur = d * tr + bl * trm + bu * trp;
                const double ui = d * ti + bl * tim + bu * tip;
                const double f = h / (double)m;
                tr = f * ui;        // -i f (ur + i ui)
                ti = -f * ur;
                sr += tr;
                si += ti;
            }
            vr = sr;
            vi = si;
        }
        tprev = times[x];
        double sn, cs;
        sincos(sigma * times[x], &sn, &cs);     // exp(-i sigma t) = cs - i sn
        const double cr = vr * cs + vi * sn, ci = vi * cs - vr * sn;
        if (!isfinite(cr) || !isfinite(ci)) bad = 1;
        st->coef[x][2 * r] = in ? cr : 0.0;
        st->coef[x][2 * r + 1] = in ? ci : 0.0;
        lastr = cr;
        lasti = ci;
    }
    const int fail = __any(bad);
    const double cr = lane_read(lastr, k - 1), ci = lane_read(lasti, k - 1);
    if (r == 0) {
        st->err_est = st->broken ? 0.0 : st->beta[k] * sqrt(cr * cr + ci * ci);
        st->exp_fail = fail;
        st->keff_min = min(st->keff_min, k);
        st->any_break = st->any_break | st->broken;
    }
}

// ---------------------------------------------------------------------------------------
// Ground-state targeting (the same Lanczos basis, with the lowest eigenpair of T in place of
// the exponential): one wavefront per problem.  The lowest eigenvalue lambda of the k x k
// tridiagonal T is found by multisection of its Gershgorin interval: each round, lane l counts
// the eigenvalues below the l-th of 64 interior points (Sturm sequence of the LDL^T pivots) and
// the interval shrinks to the first gap that holds lambda, 65 times narrower.  Its eigenvector z
// then comes from three steps of inverse iteration on T - lambda, solved by Gaussian
// elimination with partial pivoting (lane 0, O(k) per solve, tiny pivots replaced by a floor).
// Output: coef[0] = z (real, unit norm; the combination gives the unit Ritz vector V z),
// eig = lambda, err_est = beta_k |z_{k-1}| (the residual norm ||H V z - lambda V z||).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_tridiag_lowest(const VecProb* vp, int* klog, int step) {
    KState* st = vp[blockIdx.x].st;
    const int r = threadIdx.x;
    const int k = st->keff;
    if (klog && r == 0) klog[step] = k > 0 ? k : 0;     // Lanczos vectors of this basis
    if (k <= 0) {
        st->coef[0][2 * r] = 0.0;
        st->coef[0][2 * r + 1] = 0.0;
        if (r == 0) {
            st->err_est = 0.0;
            st->eig = 0.0;
            st->keff_min = 0;
            st->any_break = 1;
        }
        return;
    }
    __shared__ double al[kMaxKrylov], bt[kMaxKrylov];   // alpha_i; beta_i couples i - 1 and i
    const bool in = r < k;
    const double a = in ? st->alpha[r] : 0.0;
    const double bl = (in && r >= 1) ? st->beta[r] : 0.0;
    const double bu = (r + 1 < k) ? st->beta[r + 1] : 0.0;
    al[r] = a;
    bt[r] = bl;
    const double reach = fabs(bl) + fabs(bu);
    double hi = wave_max(in ? a + reach : -INFINITY);
    double lo = -wave_max(in ? reach - a : -INFINITY);
    const double tnorm = fmax(fabs(hi), fabs(lo));
    const double pivmin = 1e-290 * fmax(1.0, tnorm * tnorm);
    __syncthreads();
    // multisection: count(x) = number of eigenvalues below x
    for (int it = 0; it < 16; ++it) {
        const double x = lo + (hi - lo) * (double)(r + 1) / 65.0;
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < k; ++i) {
            d = (al[i] - x) - (i ? bt[i] * bt[i] / d : 0.0);
            if (fabs(d) < pivmin) d = -pivmin;
            cnt += d < 0.0;
        }
        const unsigned long long m = __ballot(cnt >= 1);
        const int f = m ? __ffsll(m) - 1 : 64;     // first point above lambda (64: the top end)
        const double nlo = f == 0 ? lo : lo + (hi - lo) * (double)f / 65.0;
        const double nhi = f == 64 ? hi : lo + (hi - lo) * (double)(f + 1) / 65.0;
        lo = nlo;
        hi = nhi;
        if (hi - lo <= 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    }
    const double lam = 0.5 * (lo + hi);
    // factors of T - lam and the iterate, in LDS (lane 0 works on them serially)
    __shared__ double d[kMaxKrylov], du[kMaxKrylov], du2[kMaxKrylov], dl[kMaxKrylov], z[kMaxKrylov];
    __shared__ bool piv[kMaxKrylov];
    if (r == 0) {
        // inverse iteration: (T - lam) z = b, elimination with partial pivoting (rows i, i + 1)
        const double floor = fmax(pivmin, 2.220446049250313e-16 * tnorm);
        for (int i = 0; i < k; ++i) {
            d[i] = al[i] - lam;
            du[i] = i + 1 < k ? bt[i + 1] : 0.0;
            dl[i] = i + 1 < k ? bt[i + 1] : 0.0;
            du2[i] = 0.0;
            z[i] = 1.0;
        }
        for (int i = 0; i + 1 < k; ++i) {
            if (fabs(d[i]) >= fabs(dl[i])) {
                piv[i] = false;
                if (fabs(d[i]) < floor) d[i] = floor;
                const double f = dl[i] / d[i];
                dl[i] = f;
                d[i + 1] -= f * du[i];
            } else {
                piv[i] = true;
                const double f = d[i] / dl[i];
                d[i] = dl[i];
                dl[i] = f;
                const double t = du[i];
                du[i] = d[i + 1];
                d[i + 1] = t - f * d[i + 1];
                if (i + 2 < k) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du[i + 1];
                }
            }
        }
        if (fabs(d[k - 1]) < floor) d[k - 1] = floor;
        for (int it = 0; it < 3; ++it) {
            for (int i = 0; i + 1 < k; ++i) {       // apply the row operations to z
                if (piv[i]) {
                    const double t = z[i];
                    z[i] = z[i + 1];
                    z[i + 1] = t - dl[i] * z[i + 1];
                } else {
                    z[i + 1] -= dl[i] * z[i];
                }
            }
            for (int i = k - 1; i >= 0; --i) {     // back substitution with U (three diagonals)
                double t = z[i];
                if (i + 1 < k) t -= du[i] * z[i + 1];
                if (i + 2 < k) t -= du2[i] * z[i + 2];
                z[i] = t / d[i];
            }
            double nrm = 0.0, big = 0.0;
            int ib = 0;
            for (int i = 0; i < k; ++i) {
                nrm += z[i] * z[i];
                if (fabs(z[i]) > big) {
                    big = fabs(z[i]);
                    ib = i;
                }
            }
            const double s = (z[ib] < 0.0 ? -1.0 : 1.0) / sqrt(nrm);   // largest entry positive
            for (int i = 0; i < k; ++i) z[i] *= s;
        }
        st->eig = lam;
        st->err_est = st->broken ? 0.0 : fabs(st->beta[k] * z[k - 1]);
        st->exp_fail = !isfinite(lam) || !isfinite(z[k - 1]);
        st->keff_min = min(st->keff_min, k);
        st->any_break = st->any_break | st->broken;
    }
    __syncthreads();
    st->coef[0][2 * r] = in ? z[r] : 0.0;
    st->coef[0][2 * r + 1] = 0.0;
}

// ---------------------------------------------------------------------------------------
// combine: y_x = sum_{c < keff} coef_x[c] scale_c u_c for x < ntimes.  With chain != 0 the
// single output is slot 0 itself (in place) and its norm seeds the next step.  Outputs of a
// batch come from the table yst[problem * kMaxTimes + x].  Without chaining a pass may give
// each problem mult blocks per block of the other passes (no partial sums to collect).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_combine(const VecProb* vp, const int* bmap,
                                                         int mult, double* y0, double* y1,
                                                         double* y2, double* y3,
                                                         double* const* yst, int ntimes,
                                                         int chain) {
    const Where W = locate(vp, bmap, mult);
    const KState* st = W.p.st;
    __shared__ double cs[kMaxTimes][2 * kMaxKrylov];
    const int k = st->keff;
    for (int idx = threadIdx.x; idx < ntimes * k; idx += blockDim.x) {
        const int x = idx / k, c = idx % k;
        cs[x][2 * c] = st->coef[x][2 * c] * st->scale[c];
        cs[x][2 * c + 1] = st->coef[x][2 * c + 1] * st->scale[c];
    }
    __syncthreads();
    double* ys[kMaxTimes];
    if (chain) {
        ys[0] = W.p.V;
        ys[1] = ys[2] = ys[3] = nullptr;
    } else if (yst) {
#pragma unroll
        for (int x = 0; x < kMaxTimes; ++x) ys[x] = yst[W.prob * kMaxTimes + x];
    } else {
        ys[0] = y0;
        ys[1] = y1;
        ys[2] = y2;
        ys[3] = y3;
    }
    const double* V = W.p.V;
    const int64_t n = W.p.n, vstride = W.p.vstride;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)W.nbt * blockDim.x;
    for (int64_t i = (int64_t)W.lb * blockDim.x + threadIdx.x; i < n; i += stride) {
        double yr[kMaxTimes] = {0.0, 0.0, 0.0, 0.0}, yi[kMaxTimes] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
        for (int c = 0; c < k; ++c) {
            const double* u = V + (int64_t)c * vstride;
            const double ur = ldv(u, i), ui = ldv(u, n + i);
#pragma unroll
            for (int x = 0; x < kMaxTimes; ++x) {
                if (x < ntimes) {
                    const double cr = cs[x][2 * c], ci = cs[x][2 * c + 1];
                    yr[x] += cr * ur - ci * ui;
                    yi[x] += cr * ui + ci * ur;
                }
            }
        }
#pragma unroll
        for (int x = 0; x < kMaxTimes; ++x) {
            if (x < ntimes) {
                ys[x][i] = yr[x];
                ys[x][n + i] = yi[x];
            }
        }
        acc[0] += yr[0] * yr[0] + yi[0] * yi[0];
    }
    if (chain) block_partials<1>(acc, W.p.part, W.lb);
}

__global__ __launch_bounds__(kVecThreads) void k_fin_chain(const VecProb* vp) {
    const VecProb P = vp[blockIdx.x];
    __shared__ double tot[1];
    final_sums<1>(P.part, P.nb, tot);
    if (threadIdx.x == 0) begin_step(P.st, tot[0], P.st->kdim);
}

// ---------------------------------------------------------------------------------------
// launchers.  vp: device table of nprob problems; bmap: block -> problem map of the nblk
// blocks of a pass (nullptr for a single problem).
// ---------------------------------------------------------------------------------------
// Blocks of a vector pass for one problem: about one element per thread (enough waves in flight
// to cover the memory latency of these streaming passes), at most kVecMaxBlocks rows of partial
// sums.
int vec_blocks(int64_t n) {
    int64_t nb = (n / 2 + kVecThreads - 1) / kVecThreads;
    if (nb < 1) nb = 1;
    if (nb > kVecMaxBlocks) nb = kVecMaxBlocks;
    return (int)nb;
}

// Blocks of the Lanczos reduction pass: kRedElems elements per thread, at most kVecMaxBlocks.
int red_blocks(int64_t n) {
    const int64_t per = (int64_t)kVecThreads * kRedElems;
    int64_t nb = (n + per - 1) / per;
    if (nb < 1) nb = 1;
    if (nb > kVecMaxBlocks) nb = kVecMaxBlocks;
    return (int)nb;
}

hipError_t launch_start(const VecGroup& g, const double* x1, const double* const* xt, int kdim,
                        int first, hipStream_t s) {
    hipLaunchKernelGGL(k_start, dim3(g.nblk), dim3(kVecThreads), 0, s, g.vp, g.bmap, x1, xt);
    hipLaunchKernelGGL(k_fin_start, dim3(g.nprob), dim3(kVecThreads), 0, s, g.vp, kdim, first);
    return hipGetLastError();
}

namespace {

typedef void (*RedFn)(const VecProb*, const int*, int, int, int, VecProb);

template <bool FIRST, bool ONE, int... I>
constexpr auto red_table(std::integer_sequence<int, I...>) {
    return std::array<RedFn, sizeof...(I)>{&k_dreduce<I, FIRST, ONE>...};
}

// [one problem][slots of the launch]
const std::array<RedFn, kDSlots + 1> kRedFirst[2] = {
    red_table<true, false>(std::make_integer_sequence<int, kDSlots + 1>{}),
    red_table<true, true>(std::make_integer_sequence<int, kDSlots + 1>{})};
const std::array<RedFn, kDSlots + 1> kRedMore[2] = {
    red_table<false, false>(std::make_integer_sequence<int, kDSlots + 1>{}),
    red_table<false, true>(std::make_integer_sequence<int, kDSlots + 1>{})};

}  // namespace

// Runs Lanczos iteration j (after the block products of slot j) on every problem of the group.
hipError_t launch_lanczos_iter(const VecGroup& g, int j, int kdim, hipStream_t s) {
    const dim3 grid(g.nblk), gridr(g.nblkr), blk(kVecThreads);
    const int nq = j > kDSlots ? (j + kDSlots - 1) / kDSlots : 1;
    const int nc0 = min(j, kDSlots);
    // one problem (no block map): its descriptor travels by value
    const int one = g.nprob == 1 && g.bmap == nullptr && g.bmapr == nullptr;
    const VecProb* vp = g.vp;
    hipLaunchKernelGGL(kRedFirst[one][nc0], gridr, blk, 0, s, vp, g.bmapr, j, 0, 0, g.one);
    for (int q = 1; q < nq; ++q) {
        const int nc = min(kDSlots, j - q * kDSlots);
        hipLaunchKernelGGL(kRedMore[one][nc], gridr, blk, 0, s, vp, g.bmapr, j, q * kDSlots, q,
                           g.one);
    }
    const dim3 grids(nq * kDVals / (kVecThreads / 64), g.nprob);
    if (one) {
        hipLaunchKernelGGL(k_dsum<true>, grids, blk, 0, s, vp, g.one);
        hipLaunchKernelGGL(k_dupdate<true>, grid, blk, 0, s, vp, g.bmap, j, kdim, nc0, g.one);
    } else {
        hipLaunchKernelGGL(k_dsum<false>, grids, blk, 0, s, vp, g.one);
        hipLaunchKernelGGL(k_dupdate<false>, grid, blk, 0, s, vp, g.bmap, j, kdim, nc0, g.one);
    }
    return hipGetLastError();
}

// klog (one problem only, else nullptr): device array receiving the Lanczos vectors of the
// basis at index step.
hipError_t launch_lowest(const VecGroup& g, int* klog, int step, hipStream_t s) {
    hipLaunchKernelGGL(k_tridiag_lowest, dim3(g.nprob), dim3(64), 0, s, g.vp, klog, step);
    return hipGetLastError();
}

hipError_t launch_tridiag(const VecGroup& g, const double* times, int ntimes, int* klog, int step,
                          hipStream_t s) {
    double t[kMaxTimes] = {0, 0, 0, 0};
    for (int i = 0; i < ntimes; ++i) t[i] = times[i];
    hipLaunchKernelGGL(k_tridiag_expm, dim3(g.nprob), dim3(64), 0, s, g.vp, t[0], t[1], t[2], t[3],
                       ntimes, klog, step);
    return hipGetLastError();
}

// Number of non-finite values among x[0 .. m) added to *count (which the caller zeroes):
// integer atomics, one per thread that found any (their sum does not depend on the order).
__global__ __launch_bounds__(kVecThreads) void k_count_nonfinite(const double* __restrict__ x,
                                                                 int64_t m, int* count) {
    int c = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride)
        c += !isfinite(x[i]);
    if (c) atomicAdd(count, c);       // only where non-finite values were found
}

hipError_t launch_count_nonfinite(const double* x, int64_t m, int* count, hipStream_t s) {
    int64_t nb = (m + kVecThreads - 1) / kVecThreads;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)nb), dim3(kVecThreads), 0, s, x, m, count);
    return hipGetLastError();
}

// ys: ntimes output pointers of a single problem, or nullptr with yst, the batch table
// [nprob][kMaxTimes].  chain: write slot 0 in place and start the next step from it.
hipError_t launch_combine(const VecGroup& g, double* const* ys, double* const* yst, int ntimes,
                          int chain, hipStream_t s) {
    double* y[kMaxTimes] = {nullptr, nullptr, nullptr, nullptr};
    if (ys)
        for (int i = 0; i < ntimes; ++i) y[i] = ys[i];
    const int mult = chain ? 1 : g.combine_mult;
    hipLaunchKernelGGL(k_combine, dim3(g.nblk * mult), dim3(kVecThreads), 0, s, g.vp,
                       g.bmap, mult, y[0], y[1], y[2], y[3], yst, ntimes,
                       chain);
    if (chain) hipLaunchKernelGGL(k_fin_chain, dim3(g.nprob), dim3(kVecThreads), 0, s, g.vp);
    return hipGetLastError();
}

}  // namespace dmrg
