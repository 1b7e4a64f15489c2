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
// Grid-wide sums are deterministic: every block of a pass writes its partial sums and a
// one-block finalise kernel adds them in a fixed order (the kernel boundary orders the two;
// no device-wide fences or atomics inside the bandwidth-bound passes).
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

// Block-level sums of NV per-thread values; writes the block partials to
// part[blockIdx.x * NV + v].
template <int NV>
__device__ __forceinline__ void block_partials(const double (&vals)[NV], double* part) {
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
        part[(int64_t)blockIdx.x * NV + v] = s;
    }
}

// Finalise kernels run as one block of kVecThreads: totals[v] = sum_b part[b * NV + v] (fixed
// order: row b in thread b, then the block reduction of block_partials; nb <= kVecThreads).
template <int NV>
__device__ void final_sums(const double* part, int nb, double* totals_lds) {
    __shared__ double red[NV][kVecThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc[NV];
    const int b = threadIdx.x < nb ? threadIdx.x : nb - 1;   // nb <= kVecThreads
    const double keep = threadIdx.x < nb ? 1.0 : 0.0;
    const double* row = part + (int64_t)b * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = row[v] * keep;
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
// start: slot 0 <- x, partial ||x||^2
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_start(const double* __restrict__ x,
                                                       double* __restrict__ u0, int64_t n,
                                                       double* part) {
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double re = x[i], im = x[n + i];
        u0[i] = re;
        u0[n + i] = im;
        acc[0] += re * re + im * im;
    }
    block_partials<1>(acc, part);
}

__global__ __launch_bounds__(kVecThreads) void k_fin_start(KState* st, const double* part, int nb,
                                                           int kdim, int first) {
    __shared__ double tot[1];
    final_sums<1>(part, nb, tot);
    if (threadIdx.x == 0) {
        begin_step(st, tot[0], kdim);
        st->err_est = 0.0;
        st->eig_fail = 0;
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
__global__ __launch_bounds__(kVecThreads) void k_project(const double* __restrict__ V,
                                                         int64_t vstride,
                                                         const double* __restrict__ w, int64_t n,
                                                         int c0, const KState* st, double* part) {
    if (st->broken) return;
    double acc[2 * NC];
#pragma unroll
    for (int c = 0; c < 2 * NC; ++c) acc[c] = 0.0;
    const double* __restrict__ V0 = V + (int64_t)c0 * vstride;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double wr = w[i], wi = w[n + i];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* u = V0 + (int64_t)c * vstride;
            const double ur = ldv(u, i), ui = ldv(u, n + i);
            acc[2 * c] += ur * wr + ui * wi;
            acc[2 * c + 1] += ur * wi - ui * wr;
        }
    }
    block_partials<2 * NC>(acc, part);
}

// h1 (which = 1) or h2 (which = 2) entries c0..c0+NC-1 = scale_c * sums; alpha_j = Re h1_j.
template <int NC>
__global__ __launch_bounds__(kVecThreads) void k_fin_project(KState* st, const double* part,
                                                             int nb, int j, int c0, int which) {
    if (st->broken) return;
    __shared__ double tot[2 * NC];
    final_sums<2 * NC>(part, nb, tot);
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
__global__ __launch_bounds__(kVecThreads) void k_reorth1(const double* V, int64_t vstride, double* w,
                                                         int64_t n, const KState* st,
                                                         double* part) {
    if (st->broken) return;
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
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
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
    block_partials<2 * NC>(acc, part);
}

// Unfused update (j+1 beyond the register capacity of k_reorth1): w <- w - sum_c h1_c v_c.
__global__ __launch_bounds__(kVecThreads) void k_update(const double* __restrict__ V,
                                                        int64_t vstride, double* __restrict__ w,
                                                        int64_t n, int j, const KState* st) {
    if (st->broken) return;
    const int nc = j + 1;
    __shared__ double hs[2 * kMaxKrylov];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double s = st->scale[c];
        hs[2 * c] = st->h1[2 * c] * s;
        hs[2 * c + 1] = st->h1[2 * c + 1] * s;
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double wr = w[i], wi = w[n + i];
        for (int c = 0; c < nc; ++c) {
            const double* u = V + (int64_t)c * vstride;
            const double ur = u[i], ui = u[n + i];
            const double hr = hs[2 * c], hi = hs[2 * c + 1];
            wr -= hr * ur - hi * ui;
            wi -= hr * ui + hi * ur;
        }
        w[i] = wr;
        w[n + i] = wi;
    }
}

// ---------------------------------------------------------------------------------------
// reorth2: u = w - sum_c h2_c v_c -> dst (slot j+1, or w itself after the last iteration),
// partial ||u||^2
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_reorth2(const double* V, int64_t vstride,
                                                         const double* w, double* dst, int64_t n,
                                                         int j, const KState* st, double* part) {
    if (st->broken) return;
    const int nc = j + 1;
    __shared__ double hs[2 * kMaxKrylov];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double s = st->scale[c];
        hs[2 * c] = st->h2[2 * c] * s;
        hs[2 * c + 1] = st->h2[2 * c + 1] * s;
    }
    __syncthreads();
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double wr = w[i], wi = w[n + i];
        for (int c = 0; c < nc; ++c) {
            const double* u = V + (int64_t)c * vstride;
            const double ur = u[i], ui = u[n + i];
            const double hr = hs[2 * c], hi = hs[2 * c + 1];
            wr -= hr * ur - hi * ui;
            wi -= hr * ui + hi * ur;
        }
        dst[i] = wr;
        dst[n + i] = wi;
        acc[0] += wr * wr + wi * wi;
    }
    block_partials<1>(acc, part);
}

// beta_{j+1} = ||u||, breakdown test beta <= 1e-12 max(1, |alpha_i|, beta_i), scale[j+1].
__global__ __launch_bounds__(kVecThreads) void k_fin_reorth2(KState* st, const double* part,
                                                             int nb, int j) {
    if (st->broken) return;
    __shared__ double tot[1];
    final_sums<1>(part, nb, tot);
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
// Tridiagonal eigen-decomposition T = S D S^T by implicit QL with shifts, in one wavefront:
// lane i holds d_i and e_i (the chase reads them with readlane, so every lane follows the same
// scalar recursion) and row i of S in LDS; then c(t_x) = beta0 S exp(-i D t_x) S^T e_1 and the
// error estimate beta_k |c_{k-1}(t_last)|.
// ---------------------------------------------------------------------------------------
namespace {

__device__ __forceinline__ double lane_get(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double pythag(double f, double g) {
    const double t = fma(f, f, g * g);
    return (t > 1e-290 && t < 1e290) ? sqrt(t) : hypot(f, g);
}

}  // namespace

__global__ __launch_bounds__(64) void k_tridiag_expm(KState* st, double t0, double t1, double t2,
                                                     double t3, int ntimes) {
    __shared__ double Z[kMaxKrylov][kMaxKrylov + 1];
    __shared__ double ecs[kMaxTimes][kMaxKrylov], esn[kMaxTimes][kMaxKrylov];
    const int r = threadIdx.x;
    const int k = st->keff;
    const double times[kMaxTimes] = {t0, t1, t2, t3};
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
    double d = (r < k) ? st->alpha[r] : 0.0;
    double e = (r + 1 < k) ? st->beta[r + 1] : 0.0;
    if (r < k)
        for (int c = 0; c < k; ++c) Z[r][c] = (c == r) ? 1.0 : 0.0;
    const double eps = 2.220446049250313e-16;
    int fail = 0;
    for (int l = 0; l < k && !fail; ++l) {
        int iter = 0;
        while (true) {
            // m = first index >= l with a negligible off-diagonal (or k-1)
            const double dn = __shfl_down(d, 1, 64);
            const bool small = (r >= l) && (r < k - 1) && (fabs(e) <= eps * (fabs(d) + fabs(dn)));
            const uint64_t mask = (uint64_t)__ballot(small || r == k - 1) >> l;
            const int m = l + __ffsll((long long)mask) - 1;
            if (m == l) break;
            if (++iter > 60) {
                fail = 1;
                break;
            }
            const double dl = lane_get(d, l), el = lane_get(e, l);
            double g = (lane_get(d, l + 1) - dl) / (2.0 * el);
            double rr = pythag(g, 1.0);
            g = lane_get(d, m) - dl + el / (g + copysign(rr, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool deflated = false;
            double carry = (r < k) ? Z[r][m] : 0.0;   // current column i+1 of this lane's row
            int i = m - 1;
            for (; i >= l; --i) {
                const double ei = lane_get(e, i);
                const double f = s * ei;
                const double b = c * ei;
                rr = pythag(f, g);
                e = (r == i + 1) ? rr : e;
                if (rr == 0.0) {          // exact deflation inside the sweep
                    const double di1 = lane_get(d, i + 1);
                    d = (r == i + 1) ? di1 - p : d;
                    e = (r == m) ? 0.0 : e;
                    deflated = true;
                    break;
                }
                const double inv = 1.0 / rr;
                s = f * inv;
                c = g * inv;
                g = lane_get(d, i + 1) - p;
                rr = (lane_get(d, i) - g) * s + 2.0 * c * b;
                p = s * rr;
                d = (r == i + 1) ? g + p : d;
                g = c * rr - b;
                if (r < k) {              // rotate columns i, i+1 of S in this lane's row
                    const double zi = Z[r][i];
                    Z[r][i + 1] = s * zi + c * carry;
                    carry = c * zi - s * carry;
                }
            }
            if (r < k) Z[r][i + 1] = carry;   // column where the sweep stopped
            if (deflated) continue;
            const double dl2 = lane_get(d, l);
            d = (r == l) ? dl2 - p : d;
            e = (r == l) ? g : e;
            e = (r == m) ? 0.0 : e;
        }
    }
    // lane q evaluates exp(-i d_q t_x) for its own eigenvalue
    if (r < k)
        for (int x = 0; x < ntimes; ++x) sincos(-d * times[x], &esn[x][r], &ecs[x][r]);
    __syncthreads();
    const double beta0 = st->beta[0];
    for (int x = 0; x < ntimes; ++x) {
        double cr = 0.0, ci = 0.0;
        if (r < k) {
            for (int q = 0; q < k; ++q) {
                const double w = Z[r][q] * Z[0][q];
                cr += w * ecs[x][q];
                ci += w * esn[x][q];
            }
        }
        st->coef[x][2 * r] = beta0 * cr;
        st->coef[x][2 * r + 1] = beta0 * ci;
    }
    __syncthreads();
    if (r == 0) {
        const int last = ntimes - 1;
        const double cr = st->coef[last][2 * (k - 1)], ci = st->coef[last][2 * (k - 1) + 1];
        st->err_est = st->broken ? 0.0 : st->beta[k] * sqrt(cr * cr + ci * ci);
        st->eig_fail = fail;
        st->keff_min = min(st->keff_min, k);
        st->any_break = st->any_break | st->broken;
    }
}

// ---------------------------------------------------------------------------------------
// combine: y_x = sum_{c < keff} coef_x[c] scale_c u_c for x < ntimes.  With chain != 0 the
// single output y_0 is written to slot 0 in place and its norm seeds the next step.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_combine(const double* V, int64_t vstride,
                                                         double* y0, double* y1, double* y2,
                                                         double* y3, int64_t n, int ntimes,
                                                         int chain, const KState* st,
                                                         double* part) {
    __shared__ double cs[kMaxTimes][2 * kMaxKrylov];
    const int k = st->keff;
    for (int idx = threadIdx.x; idx < ntimes * k; idx += blockDim.x) {
        const int x = idx / k, c = idx % k;
        cs[x][2 * c] = st->coef[x][2 * c] * st->scale[c];
        cs[x][2 * c + 1] = st->coef[x][2 * c + 1] * st->scale[c];
    }
    __syncthreads();
    double* ys[kMaxTimes] = {y0, y1, y2, y3};
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double yr[kMaxTimes] = {0.0, 0.0, 0.0, 0.0}, yi[kMaxTimes] = {0.0, 0.0, 0.0, 0.0};
        for (int c = 0; c < k; ++c) {
            const double* u = V + (int64_t)c * vstride;
            const double ur = u[i], ui = u[n + i];
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
    if (chain) block_partials<1>(acc, part);
}

__global__ __launch_bounds__(kVecThreads) void k_fin_chain(KState* st, const double* part, int nb) {
    __shared__ double tot[1];
    final_sums<1>(part, nb, tot);
    if (threadIdx.x == 0) begin_step(st, tot[0], st->kdim);
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
// Blocks of a vector pass: at most one row of partial sums per thread of the finalise block.
int vec_blocks(int64_t n) {
    int64_t nb = (n + kVecThreads - 1) / kVecThreads;
    if (nb < 1) nb = 1;
    if (nb > kVecThreads) nb = kVecThreads;
    return (int)nb;
}

hipError_t launch_start(const double* x, double* u0, int64_t n, KState* st, double* part,
                        int kdim, int first, hipStream_t s) {
    const int nb = vec_blocks(n);
    hipLaunchKernelGGL(k_start, dim3(nb), dim3(kVecThreads), 0, s, x, u0, n, part);
    hipLaunchKernelGGL(k_fin_start, dim3(1), dim3(kVecThreads), 0, s, st, part, nb, kdim, first);
    return hipGetLastError();
}

namespace {

constexpr int kProjMax = 32;     // vectors per fused projection launch
constexpr int kReorthMax = 24;   // basis size up to which reorth1 is fused

typedef void (*ProjFn)(const double*, int64_t, const double*, int64_t, int, const KState*, double*);
typedef void (*FinFn)(KState*, const double*, int, int, int, int);
typedef void (*ReoFn)(const double*, int64_t, double*, int64_t, const KState*, double*);

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

void fin_project(KState* st, const double* part, int nb, int j, int c0, int nc, int which,
                 hipStream_t s) {
    static const auto tab = fin_table(std::make_integer_sequence<int, kProjMax>{});
    hipLaunchKernelGGL(tab[nc - 1], dim3(1), dim3(kVecThreads), 0, s, st, part, nb, j, c0, which);
}

// Projection sums of w against slots [0, nc) into h1 or h2, in register-sized pieces.
void project(const double* V, int64_t vstride, const double* w, int64_t n, int j, int nc,
             int which, KState* st, double* part, hipStream_t s) {
    static const auto tab = proj_table(std::make_integer_sequence<int, kProjMax>{});
    const int nb = vec_blocks(n);
    for (int c0 = 0; c0 < nc; c0 += kProjMax) {
        const int m = min(kProjMax, nc - c0);
        hipLaunchKernelGGL(tab[m - 1], dim3(nb), dim3(kVecThreads), 0, s, V, vstride, w, n, c0, st,
                           part);
        fin_project(st, part, nb, j, c0, m, which, s);
    }
}

}  // namespace

// Runs the reduction passes of Lanczos iteration j.
hipError_t launch_lanczos_iter(double* V, int64_t vstride, double* w, int64_t n, int j, int kdim,
                               KState* st, double* part, hipStream_t s) {
    static const auto reo = reo_table(std::make_integer_sequence<int, kReorthMax>{});
    const int nb = vec_blocks(n);
    const dim3 grid(nb), blk(kVecThreads);
    const int nc = j + 1;
    // first sweep: h1 = V^H w (alpha_j = Re h1_j)
    project(V, vstride, w, n, j, nc, 1, st, part, s);
    // second sweep: w -= V h1, h2 = V^H w
    if (nc <= kReorthMax) {
        hipLaunchKernelGGL(reo[nc - 1], grid, blk, 0, s, V, vstride, w, n, st, part);
        fin_project(st, part, nb, j, 0, nc, 2, s);
    } else {
        hipLaunchKernelGGL(k_update, grid, blk, 0, s, V, vstride, w, n, j, st);
        project(V, vstride, w, n, j, nc, 2, st, part, s);
    }
    // third pass: u = w - V h2 -> slot j+1, beta_{j+1}
    double* dst = (j + 1 < kdim) ? V + (int64_t)(j + 1) * vstride : w;
    hipLaunchKernelGGL(k_reorth2, grid, blk, 0, s, V, vstride, w, dst, n, j, st, part);
    hipLaunchKernelGGL(k_fin_reorth2, dim3(1), blk, 0, s, st, part, nb, j);
    return hipGetLastError();
}

hipError_t launch_tridiag(KState* st, const double* times, int ntimes, hipStream_t s) {
    double t[kMaxTimes] = {0, 0, 0, 0};
    for (int i = 0; i < ntimes; ++i) t[i] = times[i];
    hipLaunchKernelGGL(k_tridiag_expm, dim3(1), dim3(64), 0, s, st, t[0], t[1], t[2], t[3],
                       ntimes);
    return hipGetLastError();
}

hipError_t launch_combine(const double* V, int64_t vstride, double* const* ys, int ntimes,
                          int64_t n, int chain, KState* st, double* part, hipStream_t s) {
    double* y[kMaxTimes] = {nullptr, nullptr, nullptr, nullptr};
    for (int i = 0; i < ntimes; ++i) y[i] = ys[i];
    const int nb = vec_blocks(n);
    hipLaunchKernelGGL(k_combine, dim3(nb), dim3(kVecThreads), 0, s, V, vstride, y[0], y[1], y[2],
                       y[3], n, ntimes, chain, st, part);
    if (chain) hipLaunchKernelGGL(k_fin_chain, dim3(1), dim3(kVecThreads), 0, s, st, part, nb);
    return hipGetLastError();
}

}  // namespace dmrg
