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
// Grid-wide sums are deterministic: every block writes its partial sums, the last block to
// arrive (arrival counter + device fences) adds them in a fixed order and finalises.
#include "internal.hpp"

namespace dmrg {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-level sum of nv per-thread values vals[0..nv) (compile-time NV bound, runtime nv);
// thread 0.. write block partials to part[v * gridDim.x + blockIdx.x].
template <int NV>
__device__ __forceinline__ void block_partials(const double (&vals)[NV], int nv, double* part) {
    __shared__ double red[NV][kVecThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (v < nv) {
            const double s = wave_sum(vals[v]);
            if (lane == 0) red[v][wave] = s;
        }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kVecThreads / 64; ++w) s += red[v][w];
        part[(int64_t)v * gridDim.x + blockIdx.x] = s;
    }
}

// Returns true in the last block to finish; that block then sees every partial.
__device__ __forceinline__ bool arrive_last(uint32_t* counter) {
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t prev = atomicAdd(counter, 1u);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// In the last block: totals[v] = sum over blocks of part[v * nb + b] in a fixed order.
__device__ void final_sums(const double* part, int nv, int nb, double* totals_lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int v = wave; v < nv; v += kVecThreads / 64) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += part[(int64_t)v * nb + b];
        s = wave_sum(s);
        if (lane == 0) totals_lds[v] = s;
    }
    __syncthreads();
}

}  // namespace

// ---------------------------------------------------------------------------------------
// start: slot 0 <- x, beta0 = ||x||; resets the per-step state.
//   first != 0 also resets the per-call summaries.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_start(const double* __restrict__ x,
                                                       double* __restrict__ u0, int64_t n,
                                                       KState* st, double* part, int kdim,
                                                       int first) {
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double re = x[i], im = x[n + i];
        u0[i] = re;
        u0[n + i] = im;
        acc[0] += re * re + im * im;
    }
    block_partials<1>(acc, 1, part);
    if (!arrive_last(&st->counter[0])) return;
    __shared__ double tot[1];
    final_sums(part, 1, gridDim.x, tot);
    if (threadIdx.x == 0) {
        const double b0 = sqrt(tot[0]);
        st->beta[0] = b0;
        st->bscale = 1.0;
        st->err_est = 0.0;
        st->kdim = kdim;
        st->eig_fail = 0;
        if (b0 > 0.0) {
            st->scale[0] = 1.0 / b0;
            st->keff = kdim;
            st->broken = 0;
        } else {
            st->scale[0] = 0.0;
            st->keff = 0;
            st->broken = 1;
        }
        if (first) {
            st->keff_min = kMaxKrylov + 1;
            st->any_break = 0;
            st->beta0_first = b0;
        }
        st->counter[0] = 0;
    }
}

// ---------------------------------------------------------------------------------------
// project: h1_c = scale_c * sum conj(u_c) w  for c = c0 .. c0+nc-1 (nc <= KB);
// alpha_j = Re h1_j when j lies in the range.
// ---------------------------------------------------------------------------------------
template <int KB>
__global__ __launch_bounds__(kVecThreads) void k_project(const double* __restrict__ V,
                                                         int64_t vstride,
                                                         const double* __restrict__ w,
                                                         int64_t n, int j, int c0, int nc,
                                                         KState* st, double* part) {
    if (st->broken) return;
    double acc[2 * KB];
#pragma unroll
    for (int c = 0; c < 2 * KB; ++c) acc[c] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double wr = w[i], wi = w[n + i];
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < nc) {
                const double* u = V + (int64_t)(c0 + c) * vstride;
                const double ur = u[i], ui = u[n + i];
                acc[2 * c] += ur * wr + ui * wi;
                acc[2 * c + 1] += ur * wi - ui * wr;
            }
        }
    }
    block_partials<2 * KB>(acc, 2 * nc, part);
    if (!arrive_last(&st->counter[1])) return;
    __shared__ double tot[2 * KB];
    final_sums(part, 2 * nc, gridDim.x, tot);
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double s = st->scale[c0 + c];
        st->h1[2 * (c0 + c)] = s * tot[2 * c];
        st->h1[2 * (c0 + c) + 1] = s * tot[2 * c + 1];
        if (c0 + c == j) st->alpha[j] = s * tot[2 * c];
    }
    if (threadIdx.x == 0) st->counter[1] = 0;
}

// ---------------------------------------------------------------------------------------
// reorth1: w <- w - sum_c h1_c v_c (all c <= j), then h2_c = scale_c sum conj(u_c) w.
// Fused when j+1 <= KB; the basis slice of each element is held in registers.
// ---------------------------------------------------------------------------------------
template <int KB>
__global__ __launch_bounds__(kVecThreads) void k_reorth1(const double* __restrict__ V,
                                                         int64_t vstride, double* __restrict__ w,
                                                         int64_t n, int j, KState* st,
                                                         double* part) {
    if (st->broken) return;
    const int nc = j + 1;
    __shared__ double hs[2 * KB];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double s = st->scale[c];
        hs[2 * c] = st->h1[2 * c] * s;
        hs[2 * c + 1] = st->h1[2 * c + 1] * s;
    }
    __syncthreads();
    double acc[2 * KB];
#pragma unroll
    for (int c = 0; c < 2 * KB; ++c) acc[c] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double ur[KB], ui[KB];
        double wr = w[i], wi = w[n + i];
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < nc) {
                const double* u = V + (int64_t)c * vstride;
                ur[c] = u[i];
                ui[c] = u[n + i];
                const double hr = hs[2 * c], hi = hs[2 * c + 1];
                wr -= hr * ur[c] - hi * ui[c];
                wi -= hr * ui[c] + hi * ur[c];
            }
        }
        w[i] = wr;
        w[n + i] = wi;
#pragma unroll
        for (int c = 0; c < KB; ++c) {
            if (c < nc) {
                acc[2 * c] += ur[c] * wr + ui[c] * wi;
                acc[2 * c + 1] += ur[c] * wi - ui[c] * wr;
            }
        }
    }
    block_partials<2 * KB>(acc, 2 * nc, part);
    if (!arrive_last(&st->counter[2])) return;
    __shared__ double tot[2 * KB];
    final_sums(part, 2 * nc, gridDim.x, tot);
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double s = st->scale[c];
        st->h2[2 * c] = s * tot[2 * c];
        st->h2[2 * c + 1] = s * tot[2 * c + 1];
    }
    if (threadIdx.x == 0) st->counter[2] = 0;
}

// Unfused variant of the update (for j+1 > the register capacity): w <- w - sum_c h_c v_c,
// h taken from h1 (which = 1) or h2 (which = 2); followed by k_project into h2.
__global__ __launch_bounds__(kVecThreads) void k_update(const double* __restrict__ V,
                                                        int64_t vstride, double* __restrict__ w,
                                                        int64_t n, int j, int which,
                                                        KState* st) {
    if (st->broken) return;
    const int nc = j + 1;
    __shared__ double hs[2 * kMaxKrylov];
    const double* h = which == 1 ? st->h1 : st->h2;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double s = st->scale[c];
        hs[2 * c] = h[2 * c] * s;
        hs[2 * c + 1] = h[2 * c + 1] * s;
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

// Copies h1 into h2 (used when the unfused path computed the second projection into h1).
__global__ void k_copy_h(KState* st, int nc) {
    if (st->broken) return;
    for (int c = threadIdx.x; c < 2 * nc; c += blockDim.x) st->h2[c] = st->h1[c];
}

// ---------------------------------------------------------------------------------------
// reorth2: u = w - sum_c h2_c v_c -> slot j+1 (if j+1 < kdim), beta_{j+1} = ||u||,
// breakdown test, scale[j+1].
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_reorth2(double* V, int64_t vstride,
                                                         const double* w, double* wout, int64_t n,
                                                         int j, KState* st, double* part) {
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
        wout[i] = wr;
        wout[n + i] = wi;
        acc[0] += wr * wr + wi * wi;
    }
    block_partials<1>(acc, 1, part);
    if (!arrive_last(&st->counter[3])) return;
    __shared__ double tot[1];
    final_sums(part, 1, gridDim.x, tot);
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
        st->counter[3] = 0;
    }
}

// ---------------------------------------------------------------------------------------
// Tridiagonal eigen-decomposition T = S D S^T by implicit QL with shifts (one wavefront;
// every lane runs the same scalar chase on d, e and applies the rotations to its own row of
// S), then c(t_x) = beta0 S exp(-i D t_x) S^T e_1 for the requested times and the error
// estimate beta_k |c_{k-1}(t_last)|.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_tridiag_expm(KState* st, double t0, double t1, double t2,
                                                     double t3, int ntimes) {
    __shared__ double d[kMaxKrylov], e[kMaxKrylov];
    __shared__ double Z[kMaxKrylov][kMaxKrylov + 1];
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
    if (r < k) {
        d[r] = st->alpha[r];
        e[r] = (r + 1 < k) ? st->beta[r + 1] : 0.0;
        for (int c = 0; c < k; ++c) Z[r][c] = (c == r) ? 1.0 : 0.0;
    }
    __syncthreads();
    // The chase on d and e is identical in every lane (same inputs, same arithmetic), so each
    // lane writes the shared values itself and reads back its own writes: no barrier needed.
    int fail = 0;
    for (int l = 0; l < k; ++l) {
        int iter = 0;
        while (true) {
            int m = l;
            for (; m < k - 1; ++m) {
                const double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= 2.220446049250313e-16 * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) {
                fail = 1;
                break;
            }
            // shift: eigenvalue of the leading 2x2 of the unreduced part closer to d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double rr = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + copysign(rr, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool deflated = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                rr = hypot(f, g);
                e[i + 1] = rr;
                if (rr == 0.0) {          // exact deflation inside the sweep
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = true;
                    break;
                }
                s = f / rr;
                c = g / rr;
                g = d[i + 1] - p;
                rr = (d[i] - g) * s + 2.0 * c * b;
                p = s * rr;
                d[i + 1] = g + p;
                g = c * rr - b;
                if (r < k) {              // rotate columns i, i+1 of S in this lane's row
                    const double zi = Z[r][i], zi1 = Z[r][i + 1];
                    Z[r][i + 1] = s * zi + c * zi1;
                    Z[r][i] = c * zi - s * zi1;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
        if (fail) break;
    }
    __syncthreads();
    const double beta0 = st->beta[0];
    for (int x = 0; x < ntimes; ++x) {
        double cr = 0.0, ci = 0.0;
        if (r < k) {
            for (int q = 0; q < k; ++q) {
                double sn, cs;
                sincos(-d[q] * times[x], &sn, &cs);
                const double w = Z[r][q] * Z[0][q];
                cr += w * cs;
                ci += w * sn;
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
                                                         int chain, KState* st, double* part) {
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
    if (!chain) return;
    block_partials<1>(acc, 1, part);
    if (!arrive_last(&st->counter[0])) return;
    __shared__ double tot[1];
    final_sums(part, 1, gridDim.x, tot);
    if (threadIdx.x == 0) {
        const double b0 = sqrt(tot[0]);
        st->beta[0] = b0;
        st->bscale = 1.0;
        if (b0 > 0.0) {
            st->scale[0] = 1.0 / b0;
            st->keff = st->kdim;
            st->broken = 0;
        } else {
            st->scale[0] = 0.0;
            st->keff = 0;
            st->broken = 1;
        }
        st->counter[0] = 0;
    }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
int vec_blocks(int64_t n) {
    int64_t nb = (n + 2 * kVecThreads - 1) / (2 * kVecThreads);
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    return (int)nb;
}

hipError_t launch_start(const double* x, double* u0, int64_t n, KState* st, double* part,
                        int kdim, int first, hipStream_t s) {
    hipLaunchKernelGGL(k_start, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, x, u0, n, st, part,
                       kdim, first);
    return hipGetLastError();
}

// Runs the three reduction passes of Lanczos iteration j.
hipError_t launch_lanczos_iter(double* V, int64_t vstride, double* w, int64_t n, int j, int kdim,
                               KState* st, double* part, hipStream_t s) {
    const dim3 grid(vec_blocks(n)), blk(kVecThreads);
    const int nc = j + 1;
    // first sweep: h1 = V^H w (alpha_j = Re h1_j), in register-sized pieces
    for (int c0 = 0; c0 < nc; c0 += 32) {
        const int m = min(32, nc - c0);
        if (m <= 8)
            hipLaunchKernelGGL(k_project<8>, grid, blk, 0, s, V, vstride, w, n, j, c0, m, st, part);
        else if (m <= 16)
            hipLaunchKernelGGL(k_project<16>, grid, blk, 0, s, V, vstride, w, n, j, c0, m, st, part);
        else
            hipLaunchKernelGGL(k_project<32>, grid, blk, 0, s, V, vstride, w, n, j, c0, m, st, part);
    }
    // second sweep: w -= V h1, h2 = V^H w
    if (nc <= 8) {
        hipLaunchKernelGGL(k_reorth1<8>, grid, blk, 0, s, V, vstride, w, n, j, st, part);
    } else if (nc <= 16) {
        hipLaunchKernelGGL(k_reorth1<16>, grid, blk, 0, s, V, vstride, w, n, j, st, part);
    } else if (nc <= 24) {
        hipLaunchKernelGGL(k_reorth1<24>, grid, blk, 0, s, V, vstride, w, n, j, st, part);
    } else {
        hipLaunchKernelGGL(k_update, grid, blk, 0, s, V, vstride, w, n, j, 1, st);
        for (int c0 = 0; c0 < nc; c0 += 32) {
            const int m = min(32, nc - c0);
            hipLaunchKernelGGL(k_project<32>, grid, blk, 0, s, V, vstride, w, n, -1, c0, m, st,
                               part);
        }
        hipLaunchKernelGGL(k_copy_h, dim3(1), dim3(128), 0, s, st, nc);
    }
    // third pass: u = w - V h2 -> slot j+1, beta_{j+1}
    double* dst = (j + 1 < kdim) ? V + (int64_t)(j + 1) * vstride : w;
    hipLaunchKernelGGL(k_reorth2, grid, blk, 0, s, V, vstride, w, dst, n, j, st, part);
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
    hipLaunchKernelGGL(k_combine, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, V, vstride, y[0],
                       y[1], y[2], y[3], n, ntimes, chain, st, part);
    return hipGetLastError();
}

}  // namespace dmrg
