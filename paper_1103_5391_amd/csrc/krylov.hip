// Lanczos vector kernels, tridiagonal exponential and Krylov combination (FP64, gfx950).
//
// Sec. II.A: the Lanczos recursion is started from phi itself, H ~ V^T T V, and
//   phi(t) ~ beta0 V^T S exp(-i D t) S^T e_1,     T = S D S^T.
// Storage: slot j of the basis buffer holds u_j = beta_j v_j (the vector before
// normalisation) and the state keeps scale[j] = 1/beta_j, so no separate normalisation pass
// is needed; every consumer multiplies by scale[j] on load.
//
// Per Lanczos iteration j (after w = H v_j):
//   project   h  = V^H w,           alpha_j = Re h_j                      (one pass)
//   reorth1   w1 = w - V h,         h' = V^H w1                           (one pass)
//   reorth2   u  = w1 - V h',       beta_{j+1} = ||u||, u -> slot j+1     (one pass)
// Two classical Gram-Schmidt sweeps against the whole basis.  The three-term update
// w -= alpha_j v_j + beta_j v_{j-1} is contained in the first sweep (both vectors are in the
// basis and their coefficients are exactly alpha_j and the j-1 entry of h), so it is not a
// separate pass; in exact arithmetic the result equals update-then-two-sweeps.
//
// Every kernel runs over a table of problems (one entry for a single superblock, many for a
// batch): block b of a pass works on problem bmap[b] (problem 0 when there is no map), as block
// b - b0 of that problem's nb blocks; the one-block finalise kernels run one block per problem.
// Grid-wide sums are deterministic: every block writes its partial sums and the finalise block
// adds them in a fixed order (the kernel boundary orders the two; no device-wide fences or
// atomics inside the bandwidth-bound passes).
#include <array>
#include <utility>

#include "internal.hpp"

namespace dmrg {

namespace {

typedef const double __attribute__((address_space(1)))* gcptr;

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

// Block-level sums of NV per-thread values; writes the block partials to part[lb * NV + v].
template <int NV>
__device__ __forceinline__ void block_partials(const double (&vals)[NV], double* part, int lb) {
    __shared__ double red[NV][kVecThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double s = wave_sum(vals[v]);
        if (lane == 0) red[v][wave] = s;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kVecThreads / 64; ++w) s += red[v][w];
        part[(int64_t)lb * NV + v] = s;
    }
}

// Finalise kernels run one block of kVecThreads per problem: totals[v] = sum_b part[b * NV + v]
// in a fixed order (thread t adds rows t, t + kVecThreads, ... in turn, then the block
// reduction of block_partials; nb <= kVecMaxBlocks).
template <int NV>
__device__ void final_sums(const double* part, int nb, double* totals_lds) {
    __shared__ double red[NV][kVecThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
    for (int q = 0; q < kVecMaxBlocks / kVecThreads; ++q) {
        const int b0 = q * kVecThreads + threadIdx.x;
        const int b = b0 < nb ? b0 : nb - 1;
        const double keep = b0 < nb ? 1.0 : 0.0;
        const double* row = part + (int64_t)b * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += row[v] * keep;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double t = wave_sum(acc[v]);
        if (lane == 0) red[v][wave] = t;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < NV; v += blockDim.x) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kVecThreads / 64; ++w) t += red[v][w];
        totals_lds[v] = t;
    }
    __syncthreads();
}

// Starts a Krylov step from ||x||^2: beta0, scale0, per-step flags.
__device__ void begin_step(KState* st, double norm2, int kdim) {
    const double b0 = sqrt(norm2);
    st->beta[0] = b0;
    st->bscale = 1.0;
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
// project: partials of sum conj(u_c) w for c = c0 .. c0+NC-1.  The count is a template
// parameter so the per-vector accumulators stay in registers and no load sits under a
// data-dependent branch (which would force a wait on every outstanding load).
// ---------------------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(kVecThreads) void k_project(const VecProb* vp, const int* bmap,
                                                         int c0) {
    const Where W = locate(vp, bmap, 1);
    if (W.p.st->broken) return;
    const double* __restrict__ V0 = W.p.V + (int64_t)c0 * W.p.vstride;
    const double* __restrict__ w = W.p.w;
    const int64_t n = W.p.n, vstride = W.p.vstride;
    double acc[2 * NC];
#pragma unroll
    for (int c = 0; c < 2 * NC; ++c) acc[c] = 0.0;
    const int64_t stride = (int64_t)W.nbt * blockDim.x;
    for (int64_t i = (int64_t)W.lb * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double wr = w[i], wi = w[n + i];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* u = V0 + (int64_t)c * vstride;
            const double ur = ldv(u, i), ui = ldv(u, n + i);
            acc[2 * c] += ur * wr + ui * wi;
            acc[2 * c + 1] += ur * wi - ui * wr;
        }
    }
    block_partials<2 * NC>(acc, W.p.part, W.lb);
}

// h1 (which = 1) or h2 (which = 2) entries c0..c0+NC-1 = scale_c * sums; alpha_j = Re h1_j.
template <int NC>
__global__ __launch_bounds__(kVecThreads) void k_fin_project(const VecProb* vp, int j, int c0,
                                                             int which) {
    const VecProb P = vp[blockIdx.x];
    KState* st = P.st;
    if (st->broken) return;
    __shared__ double tot[2 * NC];
    final_sums<2 * NC>(P.part, P.nb, tot);
    double* h = which == 1 ? st->h1 : st->h2;
    for (int c = threadIdx.x; c < NC; c += blockDim.x) {
        const double s = st->scale[c0 + c];
        h[2 * (c0 + c)] = s * tot[2 * c];
        h[2 * (c0 + c) + 1] = s * tot[2 * c + 1];
        if (which == 1 && c0 + c == j) st->alpha[j] = s * tot[2 * c];
    }
}

// ---------------------------------------------------------------------------------------
// reorth1: w <- w - sum_c h1_c v_c (c < NC = j+1), partials of sum conj(u_c) w.  The second
// read of each basis element comes right after the first (cache hit).
// ---------------------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(kVecThreads) void k_reorth1(const VecProb* vp, const int* bmap) {
    const Where W = locate(vp, bmap, 1);
    const KState* st = W.p.st;
    if (st->broken) return;
    const double* V = W.p.V;
    double* w = W.p.w;
    const int64_t n = W.p.n, vstride = W.p.vstride;
    __shared__ double hs[2 * NC];
    for (int c = threadIdx.x; c < NC; c += blockDim.x) {
        const double s = st->scale[c];
        hs[2 * c] = st->h1[2 * c] * s;
        hs[2 * c + 1] = st->h1[2 * c + 1] * s;
    }
    __syncthreads();
    double acc[2 * NC];
#pragma unroll
    for (int c = 0; c < 2 * NC; ++c) acc[c] = 0.0;
    const int64_t stride = (int64_t)W.nbt * blockDim.x;
    for (int64_t i = (int64_t)W.lb * blockDim.x + threadIdx.x; i < n; i += stride) {
        double wr = w[i], wi = w[n + i];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* u = V + (int64_t)c * vstride;
            const double ur = ldv(u, i), ui = ldv(u, n + i);
            const double hr = hs[2 * c], hi = hs[2 * c + 1];
            wr -= hr * ur - hi * ui;
            wi -= hr * ui + hi * ur;
        }
        w[i] = wr;
        w[n + i] = wi;
        // reload the basis slice (cache hits) instead of holding 2 NC values in registers
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* u = V + (int64_t)c * vstride;
            const double ur = ldv(u, i), ui = ldv(u, n + i);
            acc[2 * c] += ur * wr + ui * wi;
            acc[2 * c + 1] += ur * wi - ui * wr;
        }
    }
    block_partials<2 * NC>(acc, W.p.part, W.lb);
}

// Unfused update (j+1 beyond the register capacity of k_reorth1): w <- w - sum_c h1_c v_c.
__global__ __launch_bounds__(kVecThreads) void k_update(const VecProb* vp, const int* bmap, int j) {
    const Where W = locate(vp, bmap, 1);
    const KState* st = W.p.st;
    if (st->broken) return;
    const int nc = j + 1;
    const double* __restrict__ V = W.p.V;
    double* __restrict__ w = W.p.w;
    const int64_t n = W.p.n, vstride = W.p.vstride;
    __shared__ double hs[2 * kMaxKrylov];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double s = st->scale[c];
        hs[2 * c] = st->h1[2 * c] * s;
        hs[2 * c + 1] = st->h1[2 * c + 1] * s;
    }
    __syncthreads();
    const int64_t stride = (int64_t)W.nbt * blockDim.x;
    for (int64_t i = (int64_t)W.lb * blockDim.x + threadIdx.x; i < n; i += stride) {
        double wr = w[i], wi = w[n + i];
#pragma unroll 8
        for (int c = 0; c < nc; ++c) {
            const double* u = V + (int64_t)c * vstride;
            const double ur = ldv(u, i), ui = ldv(u, n + i);
            const double hr = hs[2 * c], hi = hs[2 * c + 1];
            wr -= hr * ur - hi * ui;
            wi -= hr * ui + hi * ur;
        }
        w[i] = wr;
        w[n + i] = wi;
    }
}

// ---------------------------------------------------------------------------------------
// reorth2: u = w - sum_c h2_c v_c -> slot j+1 (or w itself after the last iteration),
// partial ||u||^2
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_reorth2(const VecProb* vp, const int* bmap, int j,
                                                         int to_slot) {
    const Where W = locate(vp, bmap, 1);
    const KState* st = W.p.st;
    if (st->broken) return;
    const int nc = j + 1;
    const double* V = W.p.V;
    const double* w = W.p.w;
    double* dst = to_slot ? W.p.V + (int64_t)(j + 1) * W.p.vstride : W.p.w;
    const int64_t n = W.p.n, vstride = W.p.vstride;
    __shared__ double hs[2 * kMaxKrylov];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double s = st->scale[c];
        hs[2 * c] = st->h2[2 * c] * s;
        hs[2 * c + 1] = st->h2[2 * c + 1] * s;
    }
    __syncthreads();
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)W.nbt * blockDim.x;
    for (int64_t i = (int64_t)W.lb * blockDim.x + threadIdx.x; i < n; i += stride) {
        double wr = w[i], wi = w[n + i];
#pragma unroll 8
        for (int c = 0; c < nc; ++c) {
            const double* u = V + (int64_t)c * vstride;
            const double ur = ldv(u, i), ui = ldv(u, n + i);
            const double hr = hs[2 * c], hi = hs[2 * c + 1];
            wr -= hr * ur - hi * ui;
            wi -= hr * ui + hi * ur;
        }
        dst[i] = wr;
        dst[n + i] = wi;
        acc[0] += wr * wr + wi * wi;
    }
    block_partials<1>(acc, W.p.part, W.lb);
}

// beta_{j+1} = ||u||, breakdown test beta <= 1e-12 max(1, |alpha_i|, beta_i), scale[j+1].
__global__ __launch_bounds__(kVecThreads) void k_fin_reorth2(const VecProb* vp, int j) {
    const VecProb P = vp[blockIdx.x];
    KState* st = P.st;
    if (st->broken) return;
    __shared__ double tot[1];
    final_sums<1>(P.part, P.nb, tot);
    if (threadIdx.x == 0) {
        const double beta = sqrt(tot[0]);
        st->beta[j + 1] = beta;
        double sc = fmax(st->bscale, fabs(st->alpha[j]));
        if (j > 0) sc = fmax(sc, st->beta[j]);
        st->bscale = sc;
        if (j < st->kdim - 1) {
            if (beta <= 1e-12 * sc) {
                st->broken = 1;
                st->keff = j + 1;
            } else {
                st->scale[j + 1] = 1.0 / beta;
            }
        } else {
            st->keff = st->kdim;
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
                                                     double t2, double t3, int ntimes) {
    KState* st = vp[blockIdx.x].st;
    const int r = threadIdx.x;
    const int k = st->keff;
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
    int64_t nb = (n + kVecThreads - 1) / kVecThreads;
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

constexpr int kProjMax = 32;     // vectors per fused projection launch
constexpr int kReorthMax = 24;   // basis size up to which reorth1 is fused

typedef void (*ProjFn)(const VecProb*, const int*, int);
typedef void (*FinFn)(const VecProb*, int, int, int);
typedef void (*ReoFn)(const VecProb*, const int*);

template <int... I>
constexpr auto proj_table(std::integer_sequence<int, I...>) {
    return std::array<ProjFn, sizeof...(I)>{&k_project<I + 1>...};
}
template <int... I>
constexpr auto fin_table(std::integer_sequence<int, I...>) {
    return std::array<FinFn, sizeof...(I)>{&k_fin_project<I + 1>...};
}
template <int... I>
constexpr auto reo_table(std::integer_sequence<int, I...>) {
    return std::array<ReoFn, sizeof...(I)>{&k_reorth1<I + 1>...};
}

const auto kProjTab = proj_table(std::make_integer_sequence<int, kProjMax>{});
const auto kFinTab = fin_table(std::make_integer_sequence<int, kProjMax>{});
const auto kReoTab = reo_table(std::make_integer_sequence<int, kReorthMax>{});

// Projection sums of w against slots [0, nc) into h1 or h2, in register-sized pieces.
void project(const VecGroup& g, int j, int nc, int which, hipStream_t s) {
    for (int c0 = 0; c0 < nc; c0 += kProjMax) {
        const int m = min(kProjMax, nc - c0);
        hipLaunchKernelGGL(kProjTab[m - 1], dim3(g.nblk), dim3(kVecThreads), 0, s, g.vp, g.bmap,
                           c0);
        hipLaunchKernelGGL(kFinTab[m - 1], dim3(g.nprob), dim3(kVecThreads), 0, s, g.vp, j, c0,
                           which);
    }
}

}  // namespace

// Runs the reduction passes of Lanczos iteration j on every problem of the group.
hipError_t launch_lanczos_iter(const VecGroup& g, int j, int kdim, hipStream_t s) {
    const dim3 grid(g.nblk), blk(kVecThreads), one(g.nprob);
    const int nc = j + 1;
    // first sweep: h1 = V^H w (alpha_j = Re h1_j)
    project(g, j, nc, 1, s);
    // second sweep: w -= V h1, h2 = V^H w
    if (nc <= kReorthMax) {
        hipLaunchKernelGGL(kReoTab[nc - 1], grid, blk, 0, s, g.vp, g.bmap);
        hipLaunchKernelGGL(kFinTab[nc - 1], one, blk, 0, s, g.vp, j, 0, 2);
    } else {
        hipLaunchKernelGGL(k_update, grid, blk, 0, s, g.vp, g.bmap, j);
        project(g, j, nc, 2, s);
    }
    // third pass: u = w - V h2 -> slot j+1, beta_{j+1}
    hipLaunchKernelGGL(k_reorth2, grid, blk, 0, s, g.vp, g.bmap, j, (j + 1 < kdim) ? 1 : 0);
    hipLaunchKernelGGL(k_fin_reorth2, one, blk, 0, s, g.vp, j);
    return hipGetLastError();
}

hipError_t launch_tridiag(const VecGroup& g, const double* times, int ntimes, hipStream_t s) {
    double t[kMaxTimes] = {0, 0, 0, 0};
    for (int i = 0; i < ntimes; ++i) t[i] = times[i];
    hipLaunchKernelGGL(k_tridiag_expm, dim3(g.nprob), dim3(64), 0, s, g.vp, t[0], t[1], t[2], t[3],
                       ntimes);
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
