// Wave-function transformation (FP64, gfx950): products of complex matrices on the FP64 MFMA.
//
// Sec. II.B: when the centre moves one site to the right, a target psi on
// (A x s1) x (s2 x R) is carried to (A' x s2) x (s3 x R'') by
//   stage A   Phi[(alpha', a), beta] = sum_alpha conj(U[alpha, alpha']) psi[alpha, (a, beta)]
//             (U: the kept eigenvectors of the system's density matrix; one product per
//             sub-block (kept sector, site state a, R sector), written into the rows of the new
//             system sector that the sub-block occupies: the regrouping of s2 is the write
//             address, with no sign since the bases are normal-ordered)
//   stage B   psi'[(alpha', a), gamma] = sum_beta Phi[(alpha', a), beta] W[gamma, beta]
//             (W_r: the states of R sector r in the product basis of s3 x R'')
// Both stages are one launch over a list of 32 x 32 output tiles, one wavefront per tile, every
// vector of the call in the second grid dimension.  A tile runs 2 x 2 MFMA 16x16x4 blocks, each
// with two accumulators: Re C += Re A Re B - Im A Im B and Im C += Re A Im B + Im A Re B.
#include <algorithm>
#include <cstdint>

#include "internal.hpp"

namespace dmrg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d4u __attribute__((ext_vector_type(4), aligned(8)));   // 8-byte aligned

// Four consecutive doubles from global memory at an 8-byte aligned address.
__device__ __forceinline__ d4 ld4u(const double* p) {
    return *((const __attribute__((address_space(1))) d4u*)p);
}

// Both planes of one operand element (zero outside the matrix; imaginary part zero for real
// operands); the access mode is a template parameter.
template <int AM>
__device__ __forceinline__ void load_a(const ZTile& t, const double* __restrict__ A, int i, int k,
                                       double& re, double& im) {
    re = 0.0;
    im = 0.0;
    if (i >= t.M || k >= t.K) return;
    if constexpr (AM == ZM_COL) {
        const int64_t at = t.aoff + (int64_t)k * t.lda + i;
        re = A[at];
        im = A[at + t.aim];
    } else if constexpr (AM == ZM_CT) {
        const int64_t at = t.aoff + (int64_t)i * t.lda + k;
        re = A[at];
        im = -A[at + t.aim];
    } else if constexpr (AM == ZM_RCOL) {
        re = A[t.aoff + (int64_t)k * t.lda + i];
    } else if constexpr (AM == ZM_RT) {
        re = A[t.aoff + (int64_t)i * t.lda + k];
    } else {
        re = i == k ? 1.0 : 0.0;
    }
}

template <int BM>
__device__ __forceinline__ void load_b(const ZTile& t, const double* __restrict__ B, int k, int j,
                                       double& re, double& im) {
    re = 0.0;
    im = 0.0;
    if (j >= t.N || k >= t.K) return;
    if constexpr (BM == ZM_COL) {
        const int64_t at = t.boff + (int64_t)j * t.ldb + k;
        re = B[at];
        im = B[at + t.bim];
    } else if constexpr (BM == ZM_CT) {      // transpose (no conjugate) of a complex matrix
        const int64_t at = t.boff + (int64_t)k * t.ldb + j;
        re = B[at];
        im = B[at + t.bim];
    } else if constexpr (BM == ZM_RCOL) {
        re = B[t.boff + (int64_t)j * t.ldb + k];
    } else {
        re = B[t.boff + (int64_t)k * t.ldb + j];
    }
}

__device__ __forceinline__ d4 mma4(const double (&a)[4], const double (&b)[4], d4 c) {
#pragma unroll
    for (int u = 0; u < 4; ++u) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], c, 0, 0, 0);
    return c;
}

}  // namespace

// One wavefront per output tile; vector v = blockIdx.y.  Lane (g, r) = (lane / 16, lane % 16)
// supplies rows (columns) r of the 16-row (16-column) blocks and the K indices 4 g + u of a
// chunk of 16 (the u-th MFMA of the chunk takes index 4 g + u from lane group g, the same for
// A and B); result element (g + 4 v, r) of a 16 x 16 block is accumulator component v.  The
// operands of the next chunk are loaded while the MFMAs of the current one run.
template <int AM, int BM>
__global__ __launch_bounds__(64) void k_zgemm(const ZTile* __restrict__ tiles, ZPtrs ptr) {
    const ZTile t = tiles[blockIdx.x];
    const int v = blockIdx.y;
    const double* __restrict__ A = ptr.a[v];
    const double* __restrict__ B = ptr.b[v];
    double* __restrict__ C = ptr.c[v];
    const int lane = threadIdx.x, g = lane >> 4, r = lane & 15;
    d4 cre[2][2], cim[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            cre[mi][nj] = (d4){0.0, 0.0, 0.0, 0.0};
            cim[mi][nj] = (d4){0.0, 0.0, 0.0, 0.0};
        }
    double ar[2][2][4], ai[2][2][4], br[2][2][4], bi[2][2][4];   // [buffer][half][u]
    auto load = [&](int buf, int k0) {
        if constexpr (AM == ZM_CT && BM == ZM_COL) {
            // both operands run along K in memory: a chunk inside K is four consecutive values
            // per lane and plane, one vector load each (rows and columns outside the matrix
            // read row or column 0 and are zeroed)
            if (k0 + 16 <= t.K) {
                const int kk = k0 + 4 * g;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = t.m0 + 16 * h + r, j = t.n0 + 16 * h + r;
                    const bool oi = i < t.M, oj = j < t.N;
                    const int64_t at = t.aoff + (int64_t)(oi ? i : 0) * t.lda + kk;
                    const int64_t bt = t.boff + (int64_t)(oj ? j : 0) * t.ldb + kk;
                    const d4 are = ld4u(A + at), aim = ld4u(A + at + t.aim);
                    const d4 bre = ld4u(B + bt), bim = ld4u(B + bt + t.bim);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        ar[buf][h][u] = oi ? are[u] : 0.0;
                        ai[buf][h][u] = oi ? -aim[u] : 0.0;   // conjugate transpose
                        br[buf][h][u] = oj ? bre[u] : 0.0;
                        bi[buf][h][u] = oj ? bim[u] : 0.0;
                    }
                }
                return;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 4 * g + u;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                load_a<AM>(t, A, t.m0 + 16 * h + r, k, ar[buf][h][u], ai[buf][h][u]);
                load_b<BM>(t, B, k, t.n0 + 16 * h + r, br[buf][h][u], bi[buf][h][u]);
            }
        }
    };
    auto mma = [&](int buf) {
        double an[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < 4; ++u) an[h][u] = -ai[buf][h][u];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int nj = 0; nj < 2; ++nj) {
                cre[mi][nj] = mma4(ar[buf][mi], br[buf][nj], cre[mi][nj]);
                cre[mi][nj] = mma4(an[mi], bi[buf][nj], cre[mi][nj]);
                cim[mi][nj] = mma4(ar[buf][mi], bi[buf][nj], cim[mi][nj]);
                cim[mi][nj] = mma4(ai[buf][mi], br[buf][nj], cim[mi][nj]);
            }
    };
    if (t.K > 0) {
        load(0, 0);
        for (int k0 = 0;; k0 += 32) {
            if (k0 + 16 < t.K) load(1, k0 + 16);
            mma(0);
            if (k0 + 16 >= t.K) break;
            if (k0 + 32 < t.K) load(0, k0 + 32);
            mma(1);
            if (k0 + 32 >= t.K) break;
        }
    }
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            const int j = t.n0 + 16 * nj + r;
            if (j >= t.N) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = t.m0 + 16 * mi + g + 4 * q;
                if (i >= t.M) continue;
                const int64_t at = t.coff + (int64_t)j * t.ldc + i;
                double vr = t.alpha * cre[mi][nj][q], vi = t.alpha * cim[mi][nj][q];
                if (t.acc) {
                    vr += C[at];
                    vi += C[at + t.cim];
                }
                C[at] = vr;
                C[at + t.cim] = vi;
            }
        }
}

// Launch of one tile list whose tiles share the operand modes (am, bm).
hipError_t launch_zgemm_modes(const ZTile* t, int n, const ZPtrs& p, int nvec, int am, int bm,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(n, nvec);
#define DMRG_ZGEMM_CASE(A_, B_)                                                            \
    if (am == A_ && bm == B_) {                                                            \
        hipLaunchKernelGGL((k_zgemm<A_, B_>), grid, dim3(64), 0, s, t, p);                 \
        return hipGetLastError();                                                          \
    }
    DMRG_ZGEMM_CASE(ZM_CT, ZM_COL)        // wave-function transformation, stage A
    DMRG_ZGEMM_CASE(ZM_COL, ZM_CT)        // wave-function transformation, stage B
    DMRG_ZGEMM_CASE(ZM_COL, ZM_RT)        // local operators: right products
    DMRG_ZGEMM_CASE(ZM_COL, ZM_RCOL)
    DMRG_ZGEMM_CASE(ZM_RCOL, ZM_COL)      // local operators: left products
    DMRG_ZGEMM_CASE(ZM_RT, ZM_COL)
    DMRG_ZGEMM_CASE(ZM_ID, ZM_COL)
#undef DMRG_ZGEMM_CASE
    return hipErrorInvalidValue;
}

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

// Stage A then stage B for nvec vectors; zero_n > 0 first clears the intermediate (nvec
// consecutive pieces of zero_n doubles from pA.c[0]), for moves whose sub-blocks leave rows of
// it unwritten.
hipError_t launch_wft(const ZTile* tA, int nA, const ZPtrs& pA, const ZTile* tB, int nB,
                      const ZPtrs& pB, int nvec, int64_t zero_n, hipStream_t s) {
    if (nvec < 1 || nvec > kWftMaxVec) return hipErrorInvalidValue;
    if (zero_n > 0) {
        const int64_t tot = zero_n * nvec;
        const int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
        hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, pA.c[0], tot);
    }
    hipError_t e = launch_zgemm_modes(tA, nA, pA, nvec, ZM_CT, ZM_COL, s);
    if (e == hipSuccess) e = launch_zgemm_modes(tB, nB, pB, nvec, ZM_COL, ZM_CT, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// One list of product tiles for nvec vectors (local operators, Sec. II.B: B|psi> and the
// measured operators).
hipError_t launch_zgemm(const ZTile* t, int n, const ZPtrs& p, int nvec, int am, int bm,
                        hipStream_t s) {
    if (nvec < 1 || nvec > kWftMaxVec) return hipErrorInvalidValue;
    return launch_zgemm_modes(t, n, p, nvec, am, bm, s);
}

// Local term with monomial factors, work group (b, c) taking elements c kMonoChunk ... of source
// block b (blocks in the first grid dimension, chunks in the second): element (i, j) goes to
// (amap(i), bmap(j)) times alpha and the two factor values; the maps are one-to-one, so no two
// elements of a term meet.  Real and imaginary planes at +nx / +ny.
constexpr int64_t kMonoChunk = 2048;    // elements of a source block per work group
__global__ __launch_bounds__(256) void k_local_mono(const SJob* __restrict__ jobs,
                                                    const int* __restrict__ mapS,
                                                    const double* __restrict__ valS,
                                                    const int* __restrict__ mapE,
                                                    const double* __restrict__ valE,
                                                    const double* __restrict__ x, int64_t nx,
                                                    double* __restrict__ y, int64_t ny) {
    const SJob J = jobs[blockIdx.x];
    const int64_t cnt = (int64_t)J.d * J.e;
    const int64_t t0 = (int64_t)blockIdx.y * kMonoChunk;
    const int64_t t1 = t0 + kMonoChunk < cnt ? t0 + kMonoChunk : cnt;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
        const int i = (int)(t % J.d), j = (int)(t / J.d);
        const int io = J.amap < 0 ? i : mapS[J.amap + i];
        const int jo = J.bmap < 0 ? j : mapE[J.bmap + j];
        if (io < 0 || jo < 0) continue;
        const double sc = J.alpha * (J.amap < 0 ? 1.0 : valS[J.amap + i]) * (J.bmap < 0 ? 1.0 : valE[J.bmap + j]);
        const int64_t src = J.src + t, dst = J.dst + (int64_t)jo * J.dout + io;
        y[dst] += sc * x[src];
        y[ny + dst] += sc * x[nx + src];
    }
}

hipError_t launch_local_mono(const SJob* jobs, int njobs, int64_t maxcnt, const int* mapS,
                             const double* valS, const int* mapE, const double* valE,
                             const double* x, int64_t nx, double* y, int64_t ny, hipStream_t s) {
    if (njobs > 0 && maxcnt > 0)
        hipLaunchKernelGGL(k_local_mono, dim3(njobs, (int)((maxcnt + kMonoChunk - 1) / kMonoChunk)), dim3(256),
                           0, s, jobs, mapS, valS, mapE, valE, x, nx, y, ny);
    return hipGetLastError();
}

hipError_t launch_zero(double* x, int64_t n, hipStream_t s) {
    if (n > 0) {
        const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, x, n);
    }
    return hipGetLastError();
}

// Partial sums of <x|z> = sum conj(x) z over n complex elements (planes at +n): block b writes
// (Re, Im) of its grid-stride share to part[2 b], part[2 b + 1]; the caller adds the partials
// in order.
__global__ __launch_bounds__(256) void k_zdot(const double* __restrict__ x, const double* __restrict__ z,
                                              int64_t n, double* __restrict__ part) {
    __shared__ double sr[256], si[256];
    double ar = 0.0, ai = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double xr = x[i], xi = x[n + i], zr = z[i], zi = z[n + i];
        ar += xr * zr + xi * zi;
        ai += xr * zi - xi * zr;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sr[threadIdx.x] += sr[threadIdx.x + s];
            si[threadIdx.x] += si[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sr[0];
        part[2 * blockIdx.x + 1] = si[0];
    }
}

hipError_t launch_zdot(const double* x, const double* z, int64_t n, double* part, int nblocks,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_zdot, dim3(nblocks), dim3(256), 0, s, x, z, n, part);
    return hipGetLastError();
}

}  // namespace dmrg
