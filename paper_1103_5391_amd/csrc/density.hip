// Reduced density matrix of the time-step targets and its truncation (FP64, gfx950).
//
// Sec. II.B: the states kept for the next block are the eigenvectors of
//   rho = sum_l w_l Tr_E |phi_l><phi_l|
// with the largest eigenvalues, the targets phi_l weighted as in time-step targeting.  All
// targets lie in one (N_up, N_dn) sector, so rho is block diagonal over the system sectors p:
//   rho_p = sum_l w_l Psi_{l,p} Psi_{l,p}^H       (d_p x d_p, complex Hermitian)
// with Psi_{l,p} the d_p x e_q block of target l.  Steps:
//   k_density   rho_p in 16 x 16 tiles (one work group per tile; row panels of the blocks staged
//               through LDS, K = e_q columns per target, every target in turn)
//   k_jacobi    eigen-decomposition of every rho_p by cyclic two-sided Jacobi, one work group
//               per sector: rounds of d/2 disjoint rotations in the round-robin (circle) order,
//               each rotation the phase that makes rho_pq real times the real rotation that
//               zeroes it.  A round is one pass: the 2 x 2 block of rho at rows of pair k' and
//               columns of pair k is multiplied by U_k'^H on the left and U_k on the right, for
//               k' <= k (the block and its mirror written; rho stays Hermitian), and the columns
//               of the eigenvector matrix by U_k.  Rotations too small to matter for the
//               stopping rule are skipped with their blocks; sweeps end when the off-diagonal
//               norm is below d eps of the whole
//   k_rank      global rank of every eigenvalue (larger first; equal values by sector, then by
//               index), kept if the rank is below m
//   k_finish    per sector: eigenvalues in descending order with their eigenvectors, the number
//               kept, and the sums of all and of the kept eigenvalues (fixed-order reductions)
// The matrices live in global memory (L2-resident for the sector sizes of these workloads); the
// waves of a Jacobi work group hand them to each other through it, each wave waiting for its own
// stores to complete before the barrier that hands them over.
#include <cstdint>

#include "internal.hpp"

namespace dmrg {

namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));   // complex: (re, im)

__device__ __forceinline__ dv2 cmul(dv2 a, dv2 b) {
    return (dv2){a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ dv2 cconj(dv2 a) { return (dv2){a.x, -a.y}; }

constexpr int kJacThreads = 1024;   // threads of a Jacobi work group
constexpr int kJacBlkBatch = 2;     // rho blocks whose loads a thread issues together
constexpr int kJacVecBatch = 2;     // eigenvector items whose loads a thread issues together

// Sum over a work group of NT threads, the same value returned to every thread; fixed order.
template <int NT>
__device__ double group_sum(double v, double* scratch) {
    const int tid = threadIdx.x;
    scratch[tid] = v;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (tid < s) scratch[tid] += scratch[tid + s];
        __syncthreads();
    }
    const double out = scratch[0];
    __syncthreads();
    return out;
}

// Barrier that hands global-memory data written by the waves of the work group to the others:
// every wave first waits until its own memory operations have completed.
__device__ __forceinline__ void handover_barrier() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Right-multiplication of the row pair (x0 x1) by U = [[c, s], [-s e, c e]].
__device__ __forceinline__ void rot_right(dv2& x0, dv2& x1, double c, double sn, dv2 e) {
    const dv2 y = cmul(e, x1);
    const dv2 n0 = c * x0 - sn * y, n1 = sn * x0 + c * y;
    x0 = n0;
    x1 = n1;
}

// Left-multiplication of the column pair (x0; x1) by U^H (U as above).
__device__ __forceinline__ void rot_left(dv2& x0, dv2& x1, double c, double sn, dv2 e) {
    const dv2 y = cmul(cconj(e), x1);
    const dv2 n0 = c * x0 - sn * y, n1 = sn * x0 + c * y;
    x0 = n0;
    x1 = n1;
}

}  // namespace

// rho tiles: element (i, j) = sum_l w_l sum_c Psi_l[i, c] conj(Psi_l[j, c]), written to A
// (complex, column-major d x d at blk.aoff).  Thread (ti, tj) of the 16 x 16 work group owns
// element (i0 + ti, j0 + tj).
__global__ __launch_bounds__(256) void k_density(const DBlock* __restrict__ blks,
                                                 const DTile* __restrict__ tiles,
                                                 const double* const* __restrict__ vecs,
                                                 const double* __restrict__ weights, int nv,
                                                 int64_t n, dv2* __restrict__ A) {
    const DTile tl = tiles[blockIdx.x];
    const DBlock B = blks[tl.blk];
    const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
    __shared__ double pr[2][16][17], pi[2][16][17];   // [row panel i / j][row][column]
    const int i = tl.i0 + ti, j = tl.j0 + tj;
    double sr = 0.0, si = 0.0;
    for (int l = 0; l < nv; ++l) {
        const double* x = vecs[l];
        const double w = weights[l];
        double lr = 0.0, li = 0.0;
        for (int c0 = 0; c0 < B.e; c0 += 16) {
            // thread (ti, tj) stages element (row ti, column tj) of both panels
            const int c = c0 + tj;
            const int ri = tl.i0 + ti, rj = tl.j0 + ti;
            const bool okc = c < B.e;
            const int64_t bi = B.off + (int64_t)c * B.d + ri, bj = B.off + (int64_t)c * B.d + rj;
            pr[0][ti][tj] = (okc && ri < B.d) ? x[bi] : 0.0;
            pi[0][ti][tj] = (okc && ri < B.d) ? x[n + bi] : 0.0;
            pr[1][ti][tj] = (okc && rj < B.d) ? x[bj] : 0.0;
            pi[1][ti][tj] = (okc && rj < B.d) ? x[n + bj] : 0.0;
            __syncthreads();
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const double ar = pr[0][ti][k], ai = pi[0][ti][k];
                const double br = pr[1][tj][k], bi2 = pi[1][tj][k];
                lr += ar * br + ai * bi2;        // a conj(b)
                li += ai * br - ar * bi2;
            }
            __syncthreads();
        }
        sr += w * lr;
        si += w * li;
    }
    if (i < B.d && j < B.d) A[B.aoff + (int64_t)j * B.d + i] = (dv2){sr, si};
}

// Cyclic Jacobi on rho_p (one work group per sector): eigenvalues to ev[blk.eoff ..] (in the
// order of the diagonal), eigenvectors as the columns of V (column-major d x d at blk.aoff).
__global__ __launch_bounds__(kJacThreads) void k_jacobi(const DBlock* __restrict__ blks,
                                                        dv2* __restrict__ A, dv2* __restrict__ V,
                                                        double* __restrict__ ev, int max_sweeps) {
    const DBlock B = blks[blockIdx.x];
    const int d = B.d, tid = threadIdx.x;
    dv2* __restrict__ a = A + B.aoff;
    dv2* __restrict__ v = V + B.aoff;
    __shared__ double scratch[kJacThreads];
    __shared__ int rp[kDensMaxDim / 2], rq[kDensMaxDim / 2];
    __shared__ double rc[kDensMaxDim / 2], rs[kDensMaxDim / 2];
    __shared__ dv2 re[kDensMaxDim / 2];
    __shared__ int done;
    for (int64_t idx = tid; idx < (int64_t)d * d; idx += kJacThreads) {
        const int i = (int)(idx % d), j = (int)(idx / d);
        v[idx] = (dv2){i == j ? 1.0 : 0.0, 0.0};
    }
    const int n2 = d + (d & 1), npair = n2 / 2;
    const int ntri = npair * (npair + 1) / 2;        // blocks (k', k) with k' <= k
    const int nvit = d * npair;                      // eigenvector items (row, pair)
    handover_barrier();
    for (int sweep = 0; sweep < max_sweeps && d > 1; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int64_t idx = tid; idx < (int64_t)d * d; idx += kJacThreads) {
            const dv2 z = a[idx];
            const double m2 = z.x * z.x + z.y * z.y;
            tot += m2;
            if (idx % d != idx / d) off += m2;
        }
        off = group_sum<kJacThreads>(off, scratch);
        tot = group_sum<kJacThreads>(tot, scratch);
        // converged: the off-diagonal norm at the level of the rounding of d terms
        const double lim = fmax(1e-30, (d * 2.220446049250313e-16) * (d * 2.220446049250313e-16)) * tot;
        if (tid == 0) done = off <= lim;
        __syncthreads();
        if (done) break;
        // an element whose square is below this share of the threshold is left for later sweeps
        // (if all are, the sum of their squares is below the threshold and the next sweep stops)
        const double skip = lim / ((double)d * d);
        for (int r = 0; r < n2 - 1; ++r) {
            // circle order: position 0 fixed, positions 1 .. n2-1 rotate by r; pair k joins the
            // k-th and the (n2-1-k)-th position
            for (int k = tid; k < npair; k += kJacThreads) {
                const int pk = k == 0 ? 0 : 1 + (k - 1 + r) % (n2 - 1);
                const int k2 = n2 - 1 - k;
                const int qk = 1 + (k2 - 1 + r) % (n2 - 1);
                int p = min(pk, qk), q = max(pk, qk);
                double cs = 1.0, sn = 0.0;
                dv2 e = (dv2){1.0, 0.0};
                if (q < d) {
                    const double app = a[(int64_t)p * d + p].x, aqq = a[(int64_t)q * d + q].x;
                    const dv2 apq = a[(int64_t)q * d + p];           // row p, column q
                    const double m2 = apq.x * apq.x + apq.y * apq.y;
                    if (m2 > skip && m2 > 1e-300) {
                        const double mag = sqrt(m2);
                        const double tau = (aqq - app) / (2.0 * mag);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        cs = 1.0 / sqrt(1.0 + t * t);
                        sn = t * cs;
                        e = (dv2){apq.x / mag, -apq.y / mag};           // exp(-i phase(apq))
                    }
                } else {
                    q = -1;                                             // paired with the padding
                }
                rp[k] = p;
                rq[k] = q;
                rc[k] = cs;
                rs[k] = sn;
                re[k] = e;
            }
            __syncthreads();
            // rho blocks: rows of pair k' (kp), columns of pair k; t = k (k + 1) / 2 + k'
            for (int base = tid; base < ntri; base += kJacBlkBatch * kJacThreads) {
                dv2 x[kJacBlkBatch][4];
                int ad[kJacBlkBatch][4];                        // offsets in the sector (d <= 1024)
                int kk[kJacBlkBatch], kq[kJacBlkBatch];
#pragma unroll
                for (int u = 0; u < kJacBlkBatch; ++u) {
                    const int t = base + u * kJacThreads;
                    kk[u] = -1;
#pragma unroll
                    for (int m = 0; m < 4; ++m) ad[u][m] = -1;
                    if (t >= ntri) continue;
                    int k = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
                    while (k * (k + 1) / 2 > t) --k;
                    while ((k + 1) * (k + 2) / 2 <= t) ++k;
                    const int kp = t - k * (k + 1) / 2;
                    if (rs[k] == 0.0 && rs[kp] == 0.0) continue;
                    kk[u] = k;
                    kq[u] = kp;
                    const int r0 = rp[kp], r1 = rq[kp], c0 = rp[k], c1 = rq[k];
                    ad[u][0] = c0 * d + r0;
                    if (c1 >= 0) ad[u][1] = c1 * d + r0;
                    if (r1 >= 0) ad[u][2] = c0 * d + r1;
                    if (c1 >= 0 && r1 >= 0) ad[u][3] = c1 * d + r1;
#pragma unroll
                    for (int m = 0; m < 4; ++m) x[u][m] = ad[u][m] >= 0 ? a[ad[u][m]] : (dv2){0.0, 0.0};
                }
#pragma unroll
                for (int u = 0; u < kJacBlkBatch; ++u) {
                    const int k = kk[u];
                    if (k < 0) continue;
                    const int kp = kq[u];
                    if (rs[k] != 0.0) {                      // columns: block * U_k
                        rot_right(x[u][0], x[u][1], rc[k], rs[k], re[k]);
                        rot_right(x[u][2], x[u][3], rc[k], rs[k], re[k]);
                    }
                    if (rs[kp] != 0.0) {                     // rows: U_k'^H * block
                        rot_left(x[u][0], x[u][2], rc[kp], rs[kp], re[kp]);
                        rot_left(x[u][1], x[u][3], rc[kp], rs[kp], re[kp]);
                    }
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        if (ad[u][m] >= 0) a[ad[u][m]] = x[u][m];
                    if (kp != k) {                           // mirror block: conjugate transpose
                        const int r0 = rp[kp], r1 = rq[kp], c0 = rp[k], c1 = rq[k];
                        a[r0 * d + c0] = cconj(x[u][0]);
                        if (c1 >= 0) a[r0 * d + c1] = cconj(x[u][1]);
                        if (r1 >= 0) a[r1 * d + c0] = cconj(x[u][2]);
                        if (c1 >= 0 && r1 >= 0) a[r1 * d + c1] = cconj(x[u][3]);
                    }
                }
            }
            // eigenvectors: V <- V U, columns p, q of every pair; item = k d + i
            for (int base = tid; base < nvit; base += kJacVecBatch * kJacThreads) {
                dv2 x0[kJacVecBatch], x1[kJacVecBatch];
                int ap[kJacVecBatch], aq[kJacVecBatch];
#pragma unroll
                for (int u = 0; u < kJacVecBatch; ++u) {
                    const int t = base + u * kJacThreads;
                    ap[u] = -1;
                    if (t >= nvit) continue;
                    const int i = t % d, k = t / d;
                    if (rs[k] == 0.0) continue;
                    ap[u] = rp[k] * d + i;
                    aq[u] = rq[k] * d + i;
                    x0[u] = v[ap[u]];
                    x1[u] = v[aq[u]];
                }
#pragma unroll
                for (int u = 0; u < kJacVecBatch; ++u) {
                    if (ap[u] < 0) continue;
                    const int k = (base + u * kJacThreads) / d;
                    rot_right(x0[u], x1[u], rc[k], rs[k], re[k]);
                    v[ap[u]] = x0[u];
                    v[aq[u]] = x1[u];
                }
            }
            handover_barrier();
        }
    }
    for (int i = tid; i < d; i += kJacThreads) ev[B.eoff + i] = a[(int64_t)i * d + i].x;
}

// Global rank of eigenvalue g among all ntot: larger first, equal values by sector then index
// (the order of the flat array); kept[g] = rank < keep.
__global__ __launch_bounds__(256) void k_rank(const double* __restrict__ ev, int ntot, int keep,
                                              int* __restrict__ kept) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntot) return;
    const double x = ev[g];
    int rank = 0;
    for (int h = 0; h < ntot; ++h) {
        const double y = ev[h];
        rank += (y > x) || (y == x && h < g);
    }
    kept[g] = rank < keep;
}

// Per sector: eigenvalues in descending order (equal values by index) with their eigenvectors
// (two planes, column-major d x d at 2 blk.aoff in doubles: real parts, then imaginary parts),
// the number kept and the sums of all and of the kept eigenvalues.
__global__ __launch_bounds__(256) void k_finish(const DBlock* __restrict__ blks,
                                                const double* __restrict__ ev,
                                                const int* __restrict__ kept,
                                                const dv2* __restrict__ V,
                                                double* __restrict__ evals,
                                                double* __restrict__ evecs,
                                                int* __restrict__ nkept,
                                                double* __restrict__ sums) {
    const DBlock B = blks[blockIdx.x];
    const int d = B.d, tid = threadIdx.x;
    __shared__ double scratch[kVecThreads];
    const double* e = ev + B.eoff;
    double all = 0.0, ksum = 0.0, kc = 0.0;
    for (int i = tid; i < d; i += blockDim.x) {
        const double x = e[i];
        int r = 0;
        for (int h = 0; h < d; ++h) r += (e[h] > x) || (e[h] == x && h < i);
        evals[B.eoff + r] = x;
        const dv2* src = V + B.aoff + (int64_t)i * d;
        double* dre = evecs + 2 * B.aoff + (int64_t)r * d;
        double* dim = dre + (int64_t)d * d;
        for (int row = 0; row < d; ++row) {
            const dv2 z = src[row];
            dre[row] = z.x;
            dim[row] = z.y;
        }
        all += x;
        if (kept[B.eoff + i]) {
            ksum += x;
            kc += 1.0;
        }
    }
    all = group_sum<kVecThreads>(all, scratch);
    ksum = group_sum<kVecThreads>(ksum, scratch);
    kc = group_sum<kVecThreads>(kc, scratch);
    if (tid == 0) {
        nkept[blockIdx.x] = (int)kc;
        sums[2 * blockIdx.x] = all;
        sums[2 * blockIdx.x + 1] = ksum;
    }
}

hipError_t launch_density(const DBlock* blks, int nblk, const DTile* tiles, int ntiles,
                          const double* const* vecs, const double* weights, int nv, int64_t n,
                          void* A, void* V, double* ev, int ntot, int keep, int* kept,
                          double* evals, double* evecs, int* nkept, double* sums, hipStream_t s) {
    hipLaunchKernelGGL(k_density, dim3(ntiles), dim3(256), 0, s, blks, tiles, vecs, weights, nv, n,
                       static_cast<dv2*>(A));
    hipLaunchKernelGGL(k_jacobi, dim3(nblk), dim3(kJacThreads), 0, s, blks, static_cast<dv2*>(A),
                       static_cast<dv2*>(V), ev, kDensSweeps);
    hipLaunchKernelGGL(k_rank, dim3((ntot + 255) / 256), dim3(256), 0, s, ev, ntot, keep, kept);
    hipLaunchKernelGGL(k_finish, dim3(nblk), dim3(256), 0, s, blks, ev, kept,
                       static_cast<const dv2*>(V), evals, evecs, nkept, sums);
    return hipGetLastError();
}

}  // namespace dmrg
