// Reduced density matrix of the time-step targets and its truncation (FP64, gfx950).
//
// Sec. II.B: the states kept for the next block are the eigenvectors of
//   rho = sum_l w_l Tr_E |phi_l><phi_l|
// with the largest eigenvalues, the targets phi_l weighted as in time-step targeting.  All
// targets lie in one (N_up, N_dn) sector, so rho is block diagonal over the system sectors p:
//   rho_p = sum_l w_l Psi_{l,p} Psi_{l,p}^H       (d_p x d_p, complex Hermitian)
// with Psi_{l,p} the d_p x e_q block of target l.  Steps:
//   k_density   rho_p in 16 x 16 tiles on or below the diagonal (one wavefront per tile on the
//               FP64 matrix cores, K = e_q columns per target, every target in turn)
//   k_heig      eigen-decomposition of every rho_p up to the back-transformation, one work
//               group per sector (k_heig_r for sectors of up to 160 states, with the matrix
//               in registers during the reduction): Householder reduction to a real tridiagonal matrix T,
//               eigenvalues of T by multisection on Sturm counts, eigenvectors of T by inverse
//               iteration (no cluster of close eigenvalues larger than 8) or else by implicit QL
//               with shifts (one lane lists the rotations of the next sweep while the other
//               wavefronts apply the current one to their rows)
//   k_back_t    the compact-WY factor T of every block of reflectors, all in parallel
//   k_heig_back back-transformation by the reflectors in those blocks, several work groups per
//               sector
//   k_rank      global rank of every eigenvalue (larger first; equal values by sector, then by
//               index) in pieces over a two-dimensional grid; kept if the rank is below m
//   k_finish    per sector: eigenvalues in descending order with their eigenvectors, the number
//               kept, and the sums of all and of the kept eigenvalues (fixed-order reductions)
// The matrices live in global memory (L2-resident for the sector sizes of these workloads),
// except the matrix of the register-resident Householder reduction, the trailing matrix of the
// general one once it fits in LDS, and the columns a back-transformation work group owns; the
// waves of a work group hand global data to each other through it, each wave waiting for its
// own stores to complete before the barrier that hands them over.
#include <cstdint>

#include "internal.hpp"

namespace dmrg {

namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));   // complex: (re, im)

__device__ __forceinline__ dv2 cmul(dv2 a, dv2 b) {
    return (dv2){a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ dv2 cconj(dv2 a) { return (dv2){a.x, -a.y}; }
// 1 / x: the hardware reciprocal and one Newton step (within a few ulp)
__device__ __forceinline__ double recip(double x) {
    const double r0 = __builtin_amdgcn_rcp(x);
    return fma(fma(-x, r0, 1.0), r0, r0);
}

// 1 / x with two Newton steps (to about an ulp; the reflector's scalars)
__device__ __forceinline__ double recip2(double x) {
    const double r0 = __builtin_amdgcn_rcp(x);
    const double r1 = fma(fma(-x, r0, 1.0), r0, r0);
    return fma(fma(-x, r1, 1.0), r1, r1);
}

// 1 / sqrt(x), x > 0: the hardware reciprocal square root and two Newton steps
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return y;
}

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

}  // namespace

// rho tiles on the FP64 matrix cores: element (i, j) = sum_l w_l sum_c Psi_l[i, c]
// conj(Psi_l[j, c]), as real products of the row panels P_i, P_j (16 rows, c along K) of every
// target in turn,
//   Re rho = sum_l w_l (Re P_i Re P_j^T + Im P_i Im P_j^T),
//   Im rho = sum_l w_l (Im P_i Re P_j^T - Re P_i Im P_j^T),
// one wavefront per tile (i0, j0) with j0 <= i0: v_mfma_f64_16x16x4f64 with lane (g, r) =
// (lane div 16, lane mod 16) supplying row r of each panel at column c0 + g, the weight folded
// into P_i, and the result in lane (g, r) at row g + 4 v, column r.  A tile below the diagonal
// is also written, conjugated, at (j, i) (rho is Hermitian).  Written to A (complex,
// column-major d x d at blk.aoff).  Work group 0 also clears the per-sector flags of the
// eigen-decomposition, and all work groups clear the rank counters of k_rank.
__global__ __launch_bounds__(64) void k_density(const DBlock* __restrict__ blks,
                                                const DTile* __restrict__ tiles, const DensIn in,
                                                int nv, int64_t n, dv2* __restrict__ A,
                                                int* __restrict__ fail, int nblk,
                                                int* __restrict__ kept, int ntot) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    // the per-sector flags and the rank counters of this call start at zero
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < nblk; t += blockDim.x) fail[t] = 0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntot; t += gridDim.x * blockDim.x)
        kept[t] = 0;
    const DTile tl = tiles[blockIdx.x];
    const DBlock B = blks[tl.blk];
    const int ln = threadIdx.x, g = ln >> 4, r = ln & 15;
    const int d = B.d, e = B.e;
    const int ia = tl.i0 + r, jb = tl.j0 + r;
    const bool oka = ia < d, okb = jb < d;
    const int64_t ra = B.off + (oka ? ia : 0), rb = B.off + (okb ? jb : 0);
    d4 cre[2] = {(d4){0.0, 0.0, 0.0, 0.0}, (d4){0.0, 0.0, 0.0, 0.0}};
    d4 cim[2] = {(d4){0.0, 0.0, 0.0, 0.0}, (d4){0.0, 0.0, 0.0, 0.0}};
    // one K chunk of 4 columns (c = c0 + g) into accumulator pair q
    auto chunk = [&](double are, double aim, double bre, double bim, int q) {
        cre[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(are, bre, cre[q], 0, 0, 0);
        cre[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim, bim, cre[q], 0, 0, 0);
        cim[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim, bre, cim[q], 0, 0, 0);
        cim[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-are, bim, cim[q], 0, 0, 0);
    };
    for (int l = 0; l < nv; ++l) {
        const double* __restrict__ x = in.v[l];
        const double wa = oka ? in.w[l] : 0.0;          // rows beyond d: zero
        const double mb = okb ? 1.0 : 0.0;
        int c0 = 0;
        for (; c0 + 16 <= e; c0 += 16) {                // four whole chunks, loads first
            double v[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t cc = (int64_t)(c0 + 4 * u + g) * d;
                v[u][0] = x[ra + cc];
                v[u][1] = x[n + ra + cc];
                v[u][2] = x[rb + cc];
                v[u][3] = x[n + rb + cc];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                chunk(wa * v[u][0], wa * v[u][1], mb * v[u][2], mb * v[u][3], u & 1);
        }
        for (; c0 < e; c0 += 4) {                       // the rest, columns beyond e zero
            const int c = c0 + g;
            const bool okc = c < e;
            const int64_t cc = (int64_t)(okc ? c : 0) * d;
            const double sa = okc ? wa : 0.0, sb = okc ? mb : 0.0;
            chunk(sa * x[ra + cc], sa * x[n + ra + cc], sb * x[rb + cc], sb * x[n + rb + cc], 0);
        }
    }
    const d4 sre = cre[0] + cre[1], sim = cim[0] + cim[1];
    dv2* __restrict__ a = A + B.aoff;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = tl.i0 + g + 4 * v, j = tl.j0 + r;
        if (i < d && j < d) {
            a[(int64_t)j * d + i] = (dv2){sre[v], sim[v]};
            if (tl.i0 != tl.j0) a[(int64_t)i * d + j] = (dv2){sre[v], -sim[v]};
        }
    }
}

// Sum over the work group (NT threads) of one double, returned to every thread: shuffles
// inside each wavefront, then the wave sums in a fixed order.  red: NT / 64 doubles.
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// As wg_sum, with one barrier: the caller keeps `red` untouched until a further barrier has
// passed (so every thread has read the previous sum).
template <int NT>
__device__ __forceinline__ double wg_sum1(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    return s;
}

// The same for a complex value (red: 2 NT / 64 doubles).
template <int NT>
__device__ __forceinline__ dv2 wg_sum1c(dv2 v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[2 * (threadIdx.x >> 6)] = v.x;
        red[2 * (threadIdx.x >> 6) + 1] = v.y;
    }
    __syncthreads();
    dv2 s = (dv2){0.0, 0.0};
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += (dv2){red[2 * w], red[2 * w + 1]};
    return s;
}

constexpr int kEigThreads = 512;    // threads of an eigen-decomposition work group
constexpr int kQlMaxSweeps = 64;    // QL sweeps per eigenvalue at most
constexpr int kClusterMax = 8;      // inverse iteration when no cluster of eigenvalues is larger
constexpr double kClusterGap = 1e-5;  // eigenvalues closer than this times |T| form a cluster
constexpr int kSturmPts = 1;        // Sturm sequences one lane evaluates together in bisection
constexpr int kSturmRun = 8;        // Sturm steps whose LDS reads are issued together
constexpr int kInvRun = 8;          // rows an inverse-iteration solve loads before storing
constexpr int kInvSolves = 2;       // inverse-iteration solves per eigenvector
constexpr int kWaveCluster = 4;     // clusters of at least this many members go to a wavefront
constexpr int kHhLdsDim = 66;       // largest trailing matrix the Householder phase keeps in LDS
constexpr int kQlRun = 8;           // QL rotations whose LDS reads are issued together
constexpr int kEigChunk = 16;       // loads a thread issues together in the QL rotation pass
                                    // (their values do not depend on the stores)

constexpr int kEigThreadsR = 1024;  // threads of the register-resident eigen-decomposition
constexpr int kRegBlocks = 5;        // 32-row blocks of the matrix it holds in registers
constexpr int kRegMaxDim = 32 * kRegBlocks;   // largest sector it takes
static_assert(kRegMaxDim == kDensRegMaxDim, "register-resident limit of the planner");

// A DPP move of a double (both halves), rows ROWS only; disabled and out-of-row lanes read 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

// A DPP shift of a double within rows of 16 lanes; lanes without a source read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_shr(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sums over the 16 lanes of each DPP row, for N complex values, into every lane of the row:
// rotations by 8, 4, 2 and 1 lanes, each added.  After the rotation by r the values repeat with
// period r, so the two addends of every lane's next sum are those of its partner's, swapped, and
// all lanes of a row end with the same bits.
template <int N>
__device__ __forceinline__ void row_allsums(dv2 (&v)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) { v[q].x += dpp_shr<0x128>(v[q].x); v[q].y += dpp_shr<0x128>(v[q].y); }
#pragma unroll
    for (int q = 0; q < N; ++q) { v[q].x += dpp_shr<0x124>(v[q].x); v[q].y += dpp_shr<0x124>(v[q].y); }
#pragma unroll
    for (int q = 0; q < N; ++q) { v[q].x += dpp_shr<0x122>(v[q].x); v[q].y += dpp_shr<0x122>(v[q].y); }
#pragma unroll
    for (int q = 0; q < N; ++q) { v[q].x += dpp_shr<0x121>(v[q].x); v[q].y += dpp_shr<0x121>(v[q].y); }
}

// The value of the lane 16 apart within each group of 32 lanes (ds_swizzle in bit mode: and
// mask 0x1F, or mask 0, xor mask 0x10).
__device__ __forceinline__ double swz16(double v) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    return __hiloint2double(hi, lo);
}
// Sum over each 32-lane half of the wavefront into its last lane (31 and 63), for N values
// level by level: shifts by 1, 2, 4 and 8 lanes within each row of 16 (lane 15 of a row then
// holds the row's sum), then lane 15 of rows 0 and 2 added into rows 1 and 3.  Other lanes hold
// partial sums.
template <int N>
__device__ __forceinline__ void half_sums(double (&v)[N]) {
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_shr<0x111>(v[q]);          // row_shr:1
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_shr<0x112>(v[q]);          // row_shr:2
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_shr<0x114>(v[q]);          // row_shr:4
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_shr<0x118>(v[q]);          // row_shr:8
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += dpp_mov<0x142, 0xA>(v[q]);     // row_bcast:15, rows 1, 3
}
// half_sums of the entries from L on (the leading L entries are left as they are).
template <int L, int N>
__device__ __forceinline__ void half_sums_from(double (&v)[N]) {
#pragma unroll
    for (int q = L; q < N; ++q) v[q] += dpp_shr<0x111>(v[q]);
#pragma unroll
    for (int q = L; q < N; ++q) v[q] += dpp_shr<0x112>(v[q]);
#pragma unroll
    for (int q = L; q < N; ++q) v[q] += dpp_shr<0x114>(v[q]);
#pragma unroll
    for (int q = L; q < N; ++q) v[q] += dpp_shr<0x118>(v[q]);
#pragma unroll
    for (int q = L; q < N; ++q) v[q] += dpp_mov<0x142, 0xA>(v[q]);
}
// half_sums of the complex pairs from block lo on (lo < S, the same in every lane): the pairs
// of blocks before lo are not summed.
template <int S, int B = 0>
__device__ __forceinline__ void half_sums_active(const int lo, double (&v)[2 * S]) {
    if constexpr (B + 1 < S) {
        if (lo > B) {
            half_sums_active<S, B + 1>(lo, v);
            return;
        }
    }
    half_sums_from<2 * B>(v);
}
__device__ __forceinline__ double half_sum(double v) {
    double a[1] = {v};
    half_sums<1>(a);
    return a[0];
}

// Sum over the 64 lanes of a wavefront, the same value in every lane; waves that sum the same
// values lane for lane get the same bits (the same additions in the same order).
__device__ __forceinline__ double wave_sum(double v) {
    v = half_sum(v);
    const double lo = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 31),
                                       __builtin_amdgcn_readlane(__double2loint(v), 31));
    const double hi = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 63),
                                       __builtin_amdgcn_readlane(__double2loint(v), 63));
    return lo + hi;
}

// The value of one lane (uniform lane index) in every lane.
__device__ __forceinline__ double readlane_d(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// acc + a b and acc - a conj(b) as four fused multiply-adds each
__device__ __forceinline__ dv2 cmac(dv2 acc, dv2 a, dv2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
__device__ __forceinline__ dv2 cmsc(dv2 acc, dv2 a, dv2 b) {
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}

// Householder reduction to a real tridiagonal matrix (the arithmetic of step 1 of the general
// kernel below: the same reflectors, tau_k on the diagonal of A, v_k below the subdiagonal),
// with the lower triangle of the matrix in the registers of a work group of 1024 threads, a 32 x
// 32 grid: thread (r, c) = (tid mod 32, tid div 32) holds element (32 I + r, 32 J + c) for
// J <= I < S in slot I (I + 1) / 2 + J; entries above the diagonal and beyond d are zeros and
// stay zeros.  The update of step k is applied at once.  Step k:
//   1. the half-wave that holds column k (c = k mod 32; all its rows, in its lanes' slots of
//      block column k div 32) forms the reflector: the squared norm of x below row k + 1 by
//      DPP moves over its 32 lanes, alpha = x_{k+1} from the lane that holds it, then beta,
//      tau and the scale of v in every lane alike; lane r stores v_i for its rows i (0 outside
//      k < i < d) into vs (LDS; two buffers by the parity of k, since this half-wave starts
//      step k + 1 right after its own update of step k, while others may still read v_k), the
//      diagonal entry into dg, and tau into s_tau;
//   2. the product B v over the trailing matrix: from its slots a thread forms row sums
//      (B_ij v_j, j <= i) and column sums (conj(B_ij) v_i into entry j, i > j); each half-wave
//      stores its row of row sums (rp), and the column sums over its 32 lanes, added by DPP
//      moves, are complete (cs);
//   3. thread t adds the half-waves' rows and the column sum of entry t: w0_t = tau p_t (ps);
//   4. the waves of the vector threads (t < 32 S) form the same w0^H v (the same sums in the
//      same order), and thread t stores w_t = w0_t - (tau / 2)(w0^H v) v_t;
//   5. each thread applies B <- B - v w^H - w v^H to its slots.
// Entries at or above k enter only through v and w, which vanish there, so the stale rows and
// columns of earlier steps are never masked.  Barriers end phases 1 to 4.  Blocks of rows and
// columns wholly above k (those before (k + 1) div 32) are skipped, the column sums' DPP
// additions included.
template <int S>
__device__ __forceinline__ void hh_regs(const int d, dv2* __restrict__ a, double* __restrict__ dg,
                                        double* __restrict__ e, dv2* __restrict__ vs0,
                                        dv2* __restrict__ vs1, dv2* __restrict__ ws,
                                        dv2* __restrict__ ps, dv2* __restrict__ cs,
                                        dv2* __restrict__ rp, dv2* __restrict__ s_tau) {
    constexpr int NW = kEigThreadsR / 64, MD = 32 * S;
    const int tid = threadIdx.x, r = tid & 31, c = tid >> 5, wv = tid >> 6, ln = tid & 63;
    const dv2 z = (dv2){0.0, 0.0};
    dv2 m[S * (S + 1) / 2];
#pragma unroll
    for (int I = 0; I < S; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) {
            const int i = 32 * I + r, j = 32 * J + c;
            dv2 x = z;
            if (i < d && (I > J || r >= c)) x = a[(int64_t)j * d + i];
            m[I * (I + 1) / 2 + J] = x;
        }
    for (int k = 0; k + 1 < d; ++k) {
        dv2* __restrict__ vs = (k & 1) ? vs1 : vs0;     // v of step k (two buffers by parity)
        const int kb = k >> 5;                          // block of column k
        const int lo = (k + 1) >> 5;                    // blocks below lo hold no entry > k
        const int i1 = k + 1, I1 = i1 >> 5;
        // 1. the half-wave holding column k (c = k mod 32) forms the reflector from its slots
        if (c == (k & 31)) {
            const int h = 32 * (c & 1);                 // its first lane in the wavefront
            dv2 xr[S];                                  // column k, rows 32 I + r
#pragma unroll
            for (int I = 0; I < S; ++I) {
                xr[I] = z;
#pragma unroll
                for (int J = 0; J <= I; ++J)
                    if (J == kb && I >= kb) xr[I] = m[I * (I + 1) / 2 + J];
            }
            double part = 0.0;
            dv2 x1 = z;
#pragma unroll
            for (int I = 0; I < S; ++I) {
                const int i = 32 * I + r;
                if (i > i1) {                           // rows beyond d hold zeros
                    part = fma(xr[I].x, xr[I].x, part);
                    part = fma(xr[I].y, xr[I].y, part);
                }
                if (I == I1) x1 = xr[I];
                if (i == k) dg[k] = xr[I].x;
            }
            // |x below k + 1|^2 over the half-wave (into its lane 31), and alpha = x_{k+1}
            const double xn2 = readlane_d(half_sum(part), h + 31);
            const dv2 al = (dv2){readlane_d(x1.x, h + (i1 & 31)), readlane_d(x1.y, h + (i1 & 31))};
            dv2 sc = z, tau = z;
            double beta = al.x;
            if (!(xn2 == 0.0 && al.y == 0.0)) {
                beta = -copysign(sqrt(al.x * al.x + al.y * al.y + xn2), al.x);
                const double rb = recip2(beta);
                tau = (dv2){(beta - al.x) * rb, -al.y * rb};
                const dv2 den = (dv2){al.x - beta, al.y};               // 1 / (alpha - beta)
                const double rq = recip2(den.x * den.x + den.y * den.y);
                sc = (dv2){den.x * rq, -den.y * rq};
            }
            if (r == 0) {
                e[k] = beta;
                a[(int64_t)k * d + k] = tau;
                *s_tau = tau;
            }
#pragma unroll
            for (int I = 0; I < S; ++I) {
                if (I < lo) continue;
                const int i = 32 * I + r;
                dv2 v = z;
                if (i == i1) v = (dv2){1.0, 0.0};
                else if (i > i1 && i < d) v = cmul(xr[I], sc);
                vs[i] = v;
                if (i > i1 && i < d) a[(int64_t)k * d + i] = v;   // v_k below the subdiagonal
            }
        }
        __syncthreads();
        // 2.
        {
            dv2 pr[S];
#pragma unroll
            for (int I = 0; I < S; ++I) pr[I] = z;
#pragma unroll
            for (int J = 0; J < S; ++J) {
                if (J < lo) continue;
                const dv2 vc = vs[32 * J + c];
#pragma unroll
                for (int I = J; I < S; ++I) pr[I] = cmac(pr[I], m[I * (I + 1) / 2 + J], vc);
            }
#pragma unroll
            for (int I = 0; I < S; ++I)
                if (I >= lo) rp[(2 * wv + (ln >> 5)) * MD + 32 * I + r] = pr[I];
        }
        {
            dv2 vr[S];
            double pc[2 * S];
#pragma unroll
            for (int I = 0; I < S; ++I) vr[I] = I >= lo ? vs[32 * I + r] : z;
#pragma unroll
            for (int J = 0; J < S; ++J) {
                dv2 q = z;
                if (J >= lo) {
#pragma unroll
                    for (int I = J; I < S; ++I) {
                        // conj(B_ij) v_i; the diagonal entry counts once, in the row sums
                        const dv2 b = m[I * (I + 1) / 2 + J];
                        q = cmac(q, (I > J || r != c) ? cconj(b) : z, vr[I]);
                    }
                }
                pc[2 * J] = q.x;
                pc[2 * J + 1] = q.y;
            }
            half_sums_active<S>(lo, pc);                // blocks before lo hold zeros
#pragma unroll
            for (int J = 0; J < S; ++J)
                if (J >= lo && r == 31) cs[32 * J + c] = (dv2){pc[2 * J], pc[2 * J + 1]};
        }
        __syncthreads();
        const dv2 tau = *s_tau;
        // 3.
        if (tid < MD && tid >= 32 * lo) {
            dv2 p = cs[tid];
#pragma unroll
            for (int w = 0; w < 2 * NW; ++w) p += rp[w * MD + tid];
            ps[tid] = (tid > k && tid < d) ? cmul(tau, p) : z;
        }
        __syncthreads();
        // 4.
        if (wv < (MD + 63) / 64) {                      // the waves of the vector threads t < MD
            double sr = 0.0, si = 0.0;                  // w0^H v
            for (int i = k + 1 + ln; i < d; i += 64) {
                const dv2 w = ps[i], v = vs[i];
                sr = fma(w.x, v.x, sr);
                sr = fma(w.y, v.y, sr);
                si = fma(w.x, v.y, si);
                si = fma(-w.y, v.x, si);
            }
            sr = wave_sum(sr);
            si = wave_sum(si);
            const dv2 al2 = cmul((dv2){-0.5 * tau.x, -0.5 * tau.y}, (dv2){sr, si});
            if (tid < MD && tid >= 32 * lo) ws[tid] = cmac(ps[tid], al2, vs[tid]);
        }
        __syncthreads();
        // 5.
        {
            dv2 vr[S], wr[S];
#pragma unroll
            for (int I = 0; I < S; ++I) {
                vr[I] = I >= lo ? vs[32 * I + r] : z;
                wr[I] = I >= lo ? ws[32 * I + r] : z;
            }
#pragma unroll
            for (int J = 0; J < S; ++J) {
                if (J < lo) continue;
                const dv2 vc = vs[32 * J + c], wc = ws[32 * J + c];
#pragma unroll
                for (int I = J; I < S; ++I) {
                    if (I > J || r >= c) {
                        dv2& b = m[I * (I + 1) / 2 + J];
                        b = cmsc(b, vr[I], wc);
                        b = cmsc(b, wr[I], vc);
                    }
                }
            }
        }
    }
    if (d > 0) {
        const int k = d - 1, kb = k >> 5;
        if (r == (k & 31) && c == (k & 31)) {
#pragma unroll
            for (int I = 0; I < S; ++I)
                if (I == kb) dg[k] = m[I * (I + 1) / 2 + I].x;
        }
        if (tid == 0) e[k] = 0.0;
    }
}

// The Sturm count of T - x I (the number of negative pivots of its L D L^T, that is of the
// eigenvalues below x), with the arithmetic of the multisection rounds in heig: the hardware
// reciprocal with one Newton step, runs of kSturmRun steps without the tiny-pivot guard, a run
// that ends in a NaN taken again with it.
__device__ __forceinline__ int sturm_count(int d, const double* __restrict__ dg,
                                           const double* __restrict__ e2, double x) {
    double q = dg[0] - x;
    int cnt = q < 0.0;
    auto step = [&](double di, double ei, bool guard) {
        if (guard && fabs(q) < 1e-300) q = -1e-300;
        const double r0 = __builtin_amdgcn_rcp(q);
        const double r = fma(fma(-q, r0, 1.0), r0, r0);
        q = (di - x) - ei * r;
        cnt += q < 0.0;
    };
    int i = 1;
    for (; i + kSturmRun <= d; i += kSturmRun) {
        double dr[kSturmRun], er[kSturmRun];
#pragma unroll
        for (int t = 0; t < kSturmRun; ++t) {
            dr[t] = dg[i + t];
            er[t] = e2[i - 1 + t];
        }
        const double q0 = q;
        const int c0 = cnt;
#pragma unroll
        for (int t = 0; t < kSturmRun; ++t) step(dr[t], er[t], false);
        if (__builtin_isnan(q)) {
            q = q0;
            cnt = c0;
#pragma unroll
            for (int t = 0; t < kSturmRun; ++t) step(dr[t], er[t], true);
        }
    }
    for (; i < d; ++i) step(dg[i], e2[i - 1], true);
    return cnt;
}

// Eigen-decomposition of rho_p up to the back-transformation, one work group per sector
// (LAPACK's path for Hermitian matrices):
//   1. Householder reduction to a real tridiagonal matrix: step k takes the reflector
//      H_k = I - tau_k v_k v_k^H that maps column k below the diagonal to beta_k e_1 (beta_k
//      real) and updates the trailing matrix B <- H_k^H B H_k as B - v w^H - w v^H with
//      w = tau B v - (tau / 2)(w0^H v) v, w0 = tau B v.  v_k (v_k[0] = 1) is kept below the
//      subdiagonal of A and tau_k on its diagonal.
//   2. Eigenvalues of the tridiagonal matrix by multisection on Sturm counts.
//   3. Eigenvectors of the tridiagonal matrix into the real matrix Z: inverse iteration when no
//      cluster of close eigenvalues has more than kClusterMax members (3a), else implicit QL
//      with shifts (3b: one lane runs the scalar recurrence and lists the plane rotations of a
//      sweep while the other wavefronts apply the previous sweep to their rows of Z).
// Eigenvalues go to ev, eigenvectors to Z (row-major, or column-major after QL: bit 1 of
// fail[blk]); k_heig_back applies the reflectors.  A QL sweep count above the limit sets bit 0
// of fail[blk].
// NT threads, sectors of at most MAXD states; REG: step 1 by hh_regs (NT = kEigThreadsR).
// Bisection takes GB lanes per eigenvalue, the largest power of two up to 8 with 2 GB d <= SBT.
template <int NT, int MAXD, bool REG, int SBT = NT>
__device__ __forceinline__ void heig(const DBlock B, const int blk, dv2* __restrict__ A,
                                     double* __restrict__ Zb, double* __restrict__ Sb,
                                     double* __restrict__ ev, int* __restrict__ fail) {
    const int d = B.d, tid = threadIdx.x;
    dv2* __restrict__ a = A + B.aoff;
    double* __restrict__ Z = Zb + B.aoff;
    __shared__ double dg[MAXD], e[MAXD];
    __shared__ dv2 vv[MAXD], ww[MAXD], vv1[MAXD], ww1[MAXD];
    __shared__ dv2 pp[NT];
    __shared__ double red[3 * NT / 64];
    __shared__ int s_i0[2], s_cnt[2], s_done[2], s_path, s_nlarge;
    __shared__ double s_lo, s_hi, s_tn;
    // ---------------------------------------------------------------- 1. tridiagonal
    if constexpr (REG) {
        static_assert(NT == kEigThreadsR && MAXD % 32 == 0, "32 x 32 thread grid");
        __shared__ dv2 rp[2 * (NT / 64) * MAXD];        // row sums of the half-waves
        __shared__ dv2 ws[MAXD], s_tau;
        hh_regs<MAXD / 32>(d, a, dg, e, vv, vv1, ws, ww, ww1, rp, &s_tau);
    } else {
    __shared__ dv2 s_alpha;                             // alpha of the current reflector
    __shared__ dv2 tm[kHhLdsDim * kHhLdsDim];          // trailing matrix once it fits
    // The update of step k is applied lazily, inside step k + 1's pass over the trailing
    // matrix, which also forms that step's product B v: one read and one write of the trailing
    // matrix per step.  The pending update is kept as (v, w0, al2) with w = w0 + al2 v, in one
    // of two vector sets (step k writes set k & 1 and reads set (k - 1) & 1).  Four barriers a
    // step: the norm of the column, the reflector, the hand-over after the pass (with the
    // product's partial sums), and the inner product w0^H v.  The two sums use separate buffers,
    // each reused only after further barriers.
    // The trailing matrix is read and written through an accessor M(r, c): in place in A while
    // it is larger than kHhLdsDim, then in LDS (copied once, with the pending update not yet
    // applied), so the last steps make no round trip to L2.  The reflectors and taus always go
    // to A, where the back-transformation reads them.
    double* red2 = red + NT / 64;
    dv2 al2p = (dv2){0.0, 0.0};                         // al2 of the pending update
    auto gmat = [&](int r, int c) -> dv2& { return a[(int64_t)c * d + r]; };
    int k0 = 0, L0 = 0;                                 // LDS copy of A[k0:, k0:], stride L0
    auto lmat = [&](int r, int c) -> dv2& { return tm[(c - k0) * L0 + (r - k0)]; };
    auto step = [&](const int k, auto&& M) {
        const int m = d - k - 1;
        const int64_t ck = (int64_t)k * d;
        dv2* vc = (k & 1) ? vv1 : vv;                   // this step's v and w0
        dv2* wc = (k & 1) ? ww1 : ww;
        const dv2* vq = (k & 1) ? vv : vv1;             // pending (step k - 1), rows k .. d-1
        const dv2* wq = (k & 1) ? ww : ww1;
        const bool pend = k > 0;
        // pending correction of element (r, c) of the trailing matrix, rows/columns >= k
        auto corr = [&](int r, int c) -> dv2 {
            const dv2 vr = vq[r - k], vcn = vq[c - k];
            const dv2 wr = wq[r - k] + cmul(al2p, vr), wcn = wq[c - k] + cmul(al2p, vcn);
            return cmul(vr, cconj(wcn)) + cmul(wr, cconj(vcn));
        };
        double part = 0.0;
        for (int i = tid; i < m; i += NT) {
            dv2 x = M(k + 1 + i, k);
            if (pend) x -= corr(k + 1 + i, k);
            vc[i] = x;
            if (i > 0) part += x.x * x.x + x.y * x.y;
            else s_alpha = x;
        }
        if (tid == 0) dg[k] = M(k, k).x - (pend ? corr(k, k).x : 0.0);
        const double xn2 = wg_sum1<NT>(part, red);
        // every thread forms the reflector (the same arithmetic on the same values).  alpha
        // is read from its own slot: vc[0] is overwritten with 1 below, and a wave that reached
        // this read after wave 0's store would otherwise form its reflector from alpha = 1.
        // s_alpha is next written in the following step, after the barriers below.
        const dv2 al = s_alpha;
        dv2 tau = (dv2){0.0, 0.0}, sc = (dv2){0.0, 0.0};
        double beta = al.x;
        if (!(xn2 == 0.0 && al.y == 0.0)) {
            beta = -copysign(sqrt(al.x * al.x + al.y * al.y + xn2), al.x);
            tau = (dv2){(beta - al.x) / beta, -al.y / beta};
            const dv2 den = (dv2){al.x - beta, al.y};                   // 1 / (alpha - beta)
            const double q = den.x * den.x + den.y * den.y;
            sc = (dv2){den.x / q, -den.y / q};
        }
        if (tid == 0) {
            e[k] = beta;
            a[ck + k] = tau;                                            // tau_k on the diagonal
        }
        for (int i = tid; i < m; i += NT) {                             // own entries
            const dv2 v = i == 0 ? (dv2){1.0, 0.0} : cmul(vc[i], sc);
            vc[i] = v;
            if (i > 0) a[ck + k + 1 + i] = v;                           // v_k below the subdiagonal
        }
        __syncthreads();                                                // v complete; red read
        // pass over B = A[k+1:, k+1:]: apply the pending update, store, and form w0 = tau B v
        // (rows i, column groups g; G = 1 when a thread takes whole rows)
        const int G = m >= NT ? 1 : NT / m;
        for (int it = tid; it < m * G; it += NT) {
            const int i = it % m, g = it / m;
            dv2 acc = (dv2){0.0, 0.0};
            for (int j = g; j < m; j += G) {
                dv2& bm = M(k + 1 + i, k + 1 + j);
                dv2 b = bm;
                if (pend) {
                    b -= corr(k + 1 + i, k + 1 + j);
                    bm = b;
                }
                acc += cmul(b, vc[j]);
            }
            if (G > 1) pp[it] = acc;
            else wc[i] = acc;
        }
        handover_barrier();
        double pr = 0.0, pi = 0.0;
        for (int i = tid; i < m; i += NT) {
            dv2 acc = (dv2){0.0, 0.0};
            if (G > 1)
                for (int g = 0; g < G; ++g) acc += pp[g * m + i];
            else
                acc = wc[i];
            const dv2 w = cmul(tau, acc);
            wc[i] = w;
            const dv2 v = vc[i];                                        // conj(w) v
            pr += w.x * v.x + w.y * v.y;
            pi += w.x * v.y - w.y * v.x;
        }
        const dv2 dsum = wg_sum1c<NT>((dv2){pr, pi}, red2);
        al2p = cmul((dv2){-0.5 * tau.x, -0.5 * tau.y}, dsum);
    };
    int k = 0;
    for (; k + 1 < d && d - k > kHhLdsDim; ++k) step(k, gmat);
    bool inlds = false;
    if (k + 1 < d) {
        // the previous step's stores are complete and visible (its hand-over and sum barriers)
        k0 = k;
        L0 = d - k;
        for (int t = tid; t < L0 * L0; t += NT) {
            const int c = t / L0, r = t - c * L0;
            tm[t] = a[(int64_t)(k0 + c) * d + k0 + r];
        }
        __syncthreads();
        inlds = true;
        for (; k + 1 < d; ++k) step(k, lmat);
    }
    if (d > 0) {
        // the last diagonal element, with the update of the last step
        const int k = d - 1;
        const dv2* vq = (k & 1) ? vv : vv1;
        const dv2* wq = (k & 1) ? ww : ww1;
        dv2 c0 = (dv2){0.0, 0.0};
        if (k > 0) {
            const dv2 vr = vq[0], wr = wq[0] + cmul(al2p, vr);
            c0 = cmul(vr, cconj(wr)) + cmul(wr, cconj(vr));
        }
        if (tid == 0) {
            dg[d - 1] = (inlds ? lmat(d - 1, d - 1) : gmat(d - 1, d - 1)).x - c0.x;
            e[d - 1] = 0.0;
        }
    }
    }
    __syncthreads();
    // ---------------------------------------------------------------- 2. eigenvalues
    // Bisection on Sturm counts (the signs of the pivots of T - x I = L D L^T), one thread per
    // eigenvalue, from the Gershgorin interval to an absolute width of 2 eps |T| (|T| the
    // Gershgorin bound): the reduction to T already moves the eigenvalues by about eps |T|, so
    // narrower intervals around small eigenvalues would add rounds and no accuracy (LAPACK's
    // bisection takes the same absolute tolerance by default).
    double* e2 = reinterpret_cast<double*>(pp);         // squared subdiagonal (pp is free now)
    double* lam = reinterpret_cast<double*>(ww);        // eigenvalues, ascending
    for (int i = tid; i + 1 < d; i += NT) e2[i] = e[i] * e[i];
    if (tid == 0) {
        double lo = dg[0], hi = dg[0], tn = 0.0;
        for (int i = 0; i < d; ++i) {
            const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < d ? fabs(e[i]) : 0.0);
            lo = fmin(lo, dg[i] - r);
            hi = fmax(hi, dg[i] + r);
        }
        tn = fmax(fabs(lo), fabs(hi));
        s_lo = lo - 2.220446049250313e-16 * tn - 1e-300;
        s_hi = hi + 2.220446049250313e-16 * tn + 1e-300;
        s_tn = fmax(tn, 1e-300);
    }
    __syncthreads();
    // one shared round: the counts at NT equally spaced interior points of the interval (every
    // thread one point, the arithmetic of the rounds below), from which each eigenvalue starts:
    // the first point whose count exceeds its index and the point before it (a binary search
    // for a change of the predicate count > j, which brackets eigenvalue j whatever the counts
    // do in between)
    __shared__ int s_cnt0[NT];
    const double w0 = (s_hi - s_lo) / (NT + 1);
    s_cnt0[tid] = sturm_count(d, dg, e2, s_lo + w0 * (tid + 1));
    __syncthreads();
    {
        // GB lanes per eigenvalue (a power of two inside a wavefront), kSturmPts points per lane
        // (independent Sturm sequences interleaved in one pass over T): the lanes count at
        // GB kSturmPts interior points of the interval and keep the piece that holds the
        // eigenvalue
        // Only the whole wavefronts that hold eigenvalues take part (nact threads; lanes past
        // the last eigenvalue repeat it, so that every lane of a wave runs the same rounds).
        constexpr int P = kSturmPts;
        int GB = 1;
        while (GB < 8 && 2 * GB * d <= SBT) GB *= 2;
        const int nact = GB * d >= NT ? NT : (GB * d + 63) / 64 * 64;
        const int qb = tid % GB, jslots = nact / GB;
        const int jend = (d + jslots - 1) / jslots * jslots;
        for (int j0 = tid / GB; tid < nact && j0 < jend; j0 += jslots) {
            const int j = j0 < d ? j0 : d - 1;
            int a = -1, b = NT;                         // count(a) <= j < count(b) (virtual ends)
            while (b - a > 1) {
                const int m = (a + b) >> 1;
                if (s_cnt0[m] > j) b = m; else a = m;
            }
            double lo = a < 0 ? s_lo : s_lo + w0 * (a + 1);
            double hi = b >= NT ? s_hi : s_lo + w0 * (b + 1);
            for (int it = 0; it < 256; ++it) {
                if (hi - lo <= 4.440892098500626e-16 * s_tn) break;
                const double step = (hi - lo) / (GB * P + 1);
                double x[P], q[P];
                int cnt[P];
#pragma unroll
                for (int u = 0; u < P; ++u) {
                    x[u] = lo + step * (qb * P + u + 1);
                    q[u] = dg[0] - x[u];
                    cnt[u] = q[u] < 0.0;
                }
                // 1 / q: the hardware reciprocal and one Newton step (a few ulp; the counts then
                // place each eigenvalue within a few eps |T|)
                // a pivot q with |q| < 1e-300 is taken as -1e-300 (guarded); the unguarded step
                // meets such a pivot as a NaN (1 / 0 or an overflow), after which its count is
                // discarded and the run taken again with the guard
                auto sturm = [&](double di, double ei, bool guard) {
#pragma unroll
                    for (int u = 0; u < P; ++u) {
                        if (guard && fabs(q[u]) < 1e-300) q[u] = -1e-300;
                        const double r0 = __builtin_amdgcn_rcp(q[u]);
                        const double r = fma(fma(-q[u], r0, 1.0), r0, r0);
                        q[u] = (di - x[u]) - ei * r;
                        cnt[u] += q[u] < 0.0;
                    }
                };
                int i = 1;
                for (; i + kSturmRun <= d; i += kSturmRun) {   // LDS reads of a run issued first
                    double dr[kSturmRun], er[kSturmRun];
#pragma unroll
                    for (int t = 0; t < kSturmRun; ++t) {
                        dr[t] = dg[i + t];
                        er[t] = e2[i - 1 + t];
                    }
                    double q0[P];
                    int c0[P];
#pragma unroll
                    for (int u = 0; u < P; ++u) {
                        q0[u] = q[u];
                        c0[u] = cnt[u];
                    }
#pragma unroll
                    for (int t = 0; t < kSturmRun; ++t) sturm(dr[t], er[t], false);
                    bool bad = false;
#pragma unroll
                    for (int u = 0; u < P; ++u) bad |= __builtin_isnan(q[u]);
                    if (bad) {
#pragma unroll
                        for (int u = 0; u < P; ++u) {
                            q[u] = q0[u];
                            cnt[u] = c0[u];
                        }
#pragma unroll
                        for (int t = 0; t < kSturmRun; ++t) sturm(dr[t], er[t], true);
                    }
                }
                for (; i < d; ++i) sturm(dg[i], e2[i - 1], true);
                double nlo = lo, nhi = hi;
                bool found = false;
                for (int l = 0; l < GB; ++l) {
#pragma unroll
                    for (int u = 0; u < P; ++u) {
                        const int cu = __shfl(cnt[u], (tid & 63) - qb + l, 64);
                        const double xu = lo + step * (l * P + u + 1);
                        if (!found) {
                            if (cu > j) {
                                nhi = xu;
                                found = true;
                            } else {
                                nlo = xu;
                            }
                        }
                    }
                }
                if (!(nhi - nlo < hi - lo)) break;      // no progress at rounding level
                lo = nlo;
                hi = nhi;
            }
            if (qb == 0 && j0 < d) lam[j] = 0.5 * (lo + hi);
        }
    }
    __syncthreads();
    if (tid == 0) {                                     // largest cluster decides the path
        int run = 1, big = 1;
        for (int j = 1; j < d; ++j) {
            run = lam[j] - lam[j - 1] <= kClusterGap * s_tn ? run + 1 : 1;
            big = max(big, run);
        }
        s_path = big <= kClusterMax ? 0 : 1;
    }
    __syncthreads();
    int zr = d, zc = 1;                                 // Z(i, j) at i zr + j zc
    if (s_path == 0) {
        // ------------------------------------------------------------ 3a. inverse iteration
        // Every eigenvalue has its own thread: T - lam I = P L U (partial pivoting, pivots
        // floored at eps |T|), the factorisation fused with the forward substitution of the
        // fixed start vector, and the first solve; an eigenvalue apart from both neighbours
        // takes its remaining solves (kInvSolves in all, the vector rescaled between them) on
        // the same thread and leaves 1 / |z| in sc.  Then each cluster of close eigenvalues
        // takes its members in order (the thread of its first eigenvalue, or a wavefront for a
        // cluster of kWaveCluster or more): each vector is orthogonalised against the cluster's
        // earlier vectors (modified Gram-Schmidt) after every solve, normalised, and its sc set
        // to 1.  A last pass over all elements scales the
        // columns.  Z and the factors are row-major [i][j] (consecutive threads, consecutive
        // addresses).
        // the factors of T - lam_j I, packed so that a row takes one or two wide accesses (the
        // passes are bound by memory instructions): row i of U (1 / pivot, the superdiagonals
        // 1 and 2, an unused slot) at fu[i d + j], row i of L and the swap flag (1 where rows
        // i, i + 1 were exchanged) at fl[i d + j]; consecutive threads, consecutive records
        typedef double f4u __attribute__((ext_vector_type(4), aligned(8)));
        typedef double f2u __attribute__((ext_vector_type(2), aligned(8)));
        f4u* fu = reinterpret_cast<f4u*>(Sb + 6 * B.aoff);
        f2u* fl = reinterpret_cast<f2u*>(Sb + 6 * B.aoff + 4 * (int64_t)d * d);
        double* sc = reinterpret_cast<double*>(vv1);    // per eigenvector: 1 / |z|
        const double tiny = 2.220446049250313e-16 * s_tn;
        auto first_of_cluster = [&](int j) { return j == 0 || lam[j] - lam[j - 1] > kClusterGap * s_tn; };
        // a cluster of at least kWaveCluster members: its fourth member is close too
        static_assert(kWaveCluster == 4, "large() tests three following members");
        auto large = [&](int j0) {
            return j0 + kWaveCluster - 1 < d && !first_of_cluster(j0 + 1) &&
                   !first_of_cluster(j0 + 2) && !first_of_cluster(j0 + 3);
        };
        int* const largel = reinterpret_cast<int*>(pp);   // first members of large clusters
        if (tid == 0) s_nlarge = 0;
        __syncthreads();
        // one solve of eigenvector j from Z (times scale): P, L^-1 then U^-1; returns |z|^2
        auto backward = [&](int j) {
            // backward: U^-1, runs of kInvRun rows loaded first
            double y1 = 0.0, y2 = 0.0, nrm = 0.0;
            for (int i0 = d - 1; i0 >= 0; i0 -= kInvRun) {
                double zv[kInvRun], a0[kInvRun], a1[kInvRun], a2[kInvRun];
#pragma unroll
                for (int t = 0; t < kInvRun; ++t) {
                    const int i = max(i0 - t, 0);
                    const int64_t at = (int64_t)i * d + j;
                    zv[t] = Z[at];
                    const f4u f = fu[at];
                    a0[t] = f[0];
                    a1[t] = f[1];
                    a2[t] = f[2];
                }
#pragma unroll
                for (int t = 0; t < kInvRun; ++t) {
                    if (i0 - t < 0) break;
                    const double y = (zv[t] - a1[t] * y1 - a2[t] * y2) * a0[t];
                    Z[(int64_t)(i0 - t) * d + j] = y;
                    nrm += y * y;
                    y2 = y1;
                    y1 = y;
                }
            }
            return nrm;
        };
        auto solve = [&](int j, double scale) {
            // forward: P and L^-1 (the current entry carried in a register); a run of
            // kInvRun rows is loaded before any of it is stored (row i is stored only
            // after row i + 1 is read, so no load depends on the stores)
            double cur = scale * Z[j];
            for (int i0 = 0; i0 + 1 < d; i0 += kInvRun) {
                double zn[kInvRun], pw[kInvRun], lw[kInvRun];
#pragma unroll
                for (int t = 0; t < kInvRun; ++t) {
                    const int i = min(i0 + t, d - 2);
                    const int64_t at = (int64_t)i * d + j;
                    zn[t] = Z[at + d];
                    const f2u f = fl[at];
                    lw[t] = f[0];
                    pw[t] = f[1];
                }
#pragma unroll
                for (int t = 0; t < kInvRun; ++t) {
                    if (i0 + t + 1 >= d) break;
                    double nxt = scale * zn[t];
                    if (pw[t] != 0.0) {
                        const double tt = cur;
                        cur = nxt;
                        nxt = tt;
                    }
                    Z[(int64_t)(i0 + t) * d + j] = cur;
                    cur = nxt - lw[t] * cur;
                }
            }
            Z[(int64_t)(d - 1) * d + j] = cur;
            return backward(j);
        };
        for (int j = tid; j < d; j += NT) {
            const double x = lam[j];
            // start vector cos(0.7 i + j), by the recurrence
            // cos(a + (i + 1) b) = 2 cos(b) cos(a + i b) - cos(a + (i - 1) b) (any fixed,
            // generic vector serves; this one costs no call per element)
            const double c2 = 2.0 * cos(0.7);
            double cm = cos(j - 0.7), c0 = cos((double)j);
            auto next_start = [&]() {
                const double v = c0, cn = c2 * c0 - cm;
                cm = c0;
                c0 = cn;
                return v;
            };
            // factorisation, row by row ((dd, du) = the current row's diagonal and
            // superdiagonal), with the forward substitution P, L^-1 of the start vector (the
            // current entry carried in a register)
            double dd = dg[0] - x, du = d > 1 ? e[0] : 0.0;
            double cur = next_start();
            for (int i = 0; i + 1 < d; ++i) {
                const int64_t at = (int64_t)i * d + j;
                const double sub = e[i], nd = dg[i + 1] - x, nu = i + 2 < d ? e[i + 1] : 0.0;
                double nxt = next_start();
                double m;
                if (fabs(dd) >= fabs(sub)) {
                    const double piv = fabs(dd) >= tiny ? dd : (dd < 0.0 ? -tiny : tiny);
                    const double ip = recip(piv);
                    m = sub * ip;
                    fu[at] = (f4u){ip, du, 0.0, 0.0};
                    fl[at] = (f2u){m, 0.0};
                    dd = nd - m * du;
                    du = nu;
                } else {
                    const double is = recip(sub);
                    m = dd * is;
                    fu[at] = (f4u){is, nd, nu, 0.0};
                    fl[at] = (f2u){m, 1.0};
                    dd = du - m * nd;
                    du = -m * nu;
                    const double tt = cur;
                    cur = nxt;
                    nxt = tt;
                }
                Z[at] = cur;
                cur = nxt - m * cur;
            }
            {
                const int64_t at = (int64_t)(d - 1) * d + j;
                const double piv = fabs(dd) >= tiny ? dd : (dd < 0.0 ? -tiny : tiny);
                fu[at] = (f4u){1.0 / piv, 0.0, 0.0, 0.0};
                Z[at] = cur;
            }
            // the first solve: backward substitution U^-1
            sc[j] = 1.0 / sqrt(fmax(backward(j), 1e-300));
            if (first_of_cluster(j) && large(j)) largel[atomicAdd(&s_nlarge, 1)] = j;
            // an eigenvalue apart from both neighbours: the remaining solves now
            if (first_of_cluster(j) && (j + 1 >= d || first_of_cluster(j + 1)))
                for (int rep = 1; rep < kInvSolves; ++rep) sc[j] = 1.0 / sqrt(fmax(solve(j, sc[j]), 1e-300));
            ev[B.eoff + j] = x;
        }
        handover_barrier();
        // clusters: the thread of the first member takes the members in order, each
        // orthogonalised against the cluster's earlier vectors (modified Gram-Schmidt) after
        // every solve, as the first solve was
        auto mgs = [&](int j0, int j) {                 // returns |z_j|^2 after the projection
            double nrm = 0.0;
            for (int k = j0; k < j; ++k) {
                double dot = 0.0;
                for (int i = 0; i < d; ++i) dot += Z[(int64_t)i * d + k] * Z[(int64_t)i * d + j];
                nrm = 0.0;
                for (int i = 0; i < d; ++i) {
                    const double y = Z[(int64_t)i * d + j] - dot * Z[(int64_t)i * d + k];
                    Z[(int64_t)i * d + j] = y;
                    nrm += y * y;
                }
            }
            return nrm;
        };
        for (int j0 = tid; j0 < d; j0 += NT) {
            if (!first_of_cluster(j0) || j0 + 1 >= d || first_of_cluster(j0 + 1)) continue;
            if (large(j0)) continue;
            for (int j = j0; j < d && (j == j0 || !first_of_cluster(j)); ++j) {
                double s = sc[j];
                if (j > j0) s = 1.0 / sqrt(fmax(mgs(j0, j), 1e-300));
                for (int rep = 1; rep < kInvSolves; ++rep) {
                    double nrm = solve(j, s);
                    if (j > j0) nrm = mgs(j0, j);
                    s = 1.0 / sqrt(fmax(nrm, 1e-300));
                }
                for (int i = 0; i < d; ++i) Z[(int64_t)i * d + j] *= s;
                sc[j] = 1.0;
            }
        }
        // large clusters (the Gram-Schmidt steps grow as the square of the size, listed in
        // phase 1): one wavefront each, dealt from the last wavefront down.  Lane 0 runs the solves; the lanes share the
        // Gram-Schmidt steps (rows i = lane mod 64, sums by wave_sum, the same in every lane);
        // the fences order the lanes' global stores of Z before the other lanes' loads.
        {
            const int wv = tid >> 6, lane = tid & 63;
            auto mgsw = [&](int j0, int j) {            // |z_j|^2 after the projection
                double nrm = 0.0;
                for (int k = j0; k < j; ++k) {
                    double part = 0.0;
                    for (int i = lane; i < d; i += 64)
                        part += Z[(int64_t)i * d + k] * Z[(int64_t)i * d + j];
                    const double dot = wave_sum(part);
                    double pn = 0.0;
                    for (int i = lane; i < d; i += 64) {
                        const double y = Z[(int64_t)i * d + j] - dot * Z[(int64_t)i * d + k];
                        Z[(int64_t)i * d + j] = y;
                        pn += y * y;
                    }
                    nrm = wave_sum(pn);
                }
                return nrm;
            };
            // the list's order depends on the atomics, but every cluster takes the same
            // arithmetic on whichever wavefront runs it
            for (int q = NT / 64 - 1 - wv; q < s_nlarge; q += NT / 64) {
                const int j0 = largel[q];
                for (int j = j0; j < d && (j == j0 || !first_of_cluster(j)); ++j) {
                    double s = sc[j];
                    if (j > j0) s = 1.0 / sqrt(fmax(mgsw(j0, j), 1e-300));
                    for (int rep = 1; rep < kInvSolves; ++rep) {
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                        double nrm = 0.0;
                        if (lane == 0) nrm = solve(j, s);
                        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                        nrm = __shfl(nrm, 0, 64);
                        if (j > j0) nrm = mgsw(j0, j);
                        s = 1.0 / sqrt(fmax(nrm, 1e-300));
                    }
                    for (int i = lane; i < d; i += 64) Z[(int64_t)i * d + j] *= s;
                    if (lane == 0) sc[j] = 1.0;
                }
            }
        }
        handover_barrier();
        for (int t = tid; t < d * d; t += NT) Z[t] *= sc[t % d];
        handover_barrier();
    } else {
    zr = 1;
    zc = d;
    for (int64_t it = tid; it < (int64_t)d * d; it += NT)
        Z[it] = (it % d == it / d) ? 1.0 : 0.0;
    handover_barrier();
    // ---------------------------------------------------------------- 3b. implicit QL
    // Wavefront 0 runs the sweep recurrence (its first lane) and lists the rotations of the next
    // sweep while the other wavefronts apply the current one (two rotation lists in LDS).
    auto rcl = [&](int buf) { return buf ? reinterpret_cast<double*>(ww) : reinterpret_cast<double*>(vv); };
    auto rsl = [&](int buf) { return rcl(buf) + MAXD; };
    int l = 0, sweeps = 0;                              // scalar state (the same in every lane of wave 0)
    // wave 0: the next sweep into list buf.  All its lanes look for the end m of the unreduced
    // block together (a ballot over 64 entries at a time); lane 0 runs the recurrence and makes
    // every store.  The fence orders lane 0's stores of e and dg before the other lanes' next
    // search.
    const int lane = tid & 63;
    auto next_sweep = [&](int buf) {
        double* rc = rcl(buf);
        double* rs = rsl(buf);
        if (lane == 0) {
            s_cnt[buf] = 0;
            s_done[buf] = 0;
        }
        for (;;) {
            if (l >= d) {
                if (lane == 0) s_done[buf] = 1;
                return;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            // m: the first index >= l that is the last row or has a negligible e[m]
            int m = -1;
            for (int base = l; m < 0; base += 64) {
                const int i = base + lane;
                const bool stop = i >= d - 1 ||
                    !(fabs(e[i]) > 2.220446049250313e-16 * (fabs(dg[i]) + fabs(dg[i + 1])));
                const unsigned long long hit = __ballot(stop);
                if (hit) m = base + __builtin_ctzll(hit);
            }
            if (m == l) {
                ++l;
                sweeps = 0;
                continue;
            }
            if (++sweeps > kQlMaxSweeps) {
                if (lane == 0) {
                    fail[blk] = 1;
                    s_done[buf] = 1;
                }
                return;
            }
            if (lane != 0) return;
            // shift from the leading 2 x 2 block of the unreduced part, then chase upward
            double g = (dg[l + 1] - dg[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = dg[m] - dg[l] + e[l] / (g + copysign(r, g));
            double sn = 1.0, cs = 1.0, p = 0.0;
            int cnt = 0;
            bool early = false;
            double ei = e[m - 1], di = dg[m - 1], di1 = dg[m];      // values of the next rotation
            // rotation i reads e[i - 1] and dg[i - 1] and writes entries i + 1 and above, so
            // the values of kQlRun rotations are loaded before any of them runs
            for (int i0 = m - 1; i0 >= l && !early; i0 -= kQlRun) {
                double en[kQlRun], dn[kQlRun];
#pragma unroll
                for (int t = 0; t < kQlRun; ++t) {
                    const int i = i0 - t;
                    en[t] = i > l ? e[i - 1] : 0.0;
                    dn[t] = i > l ? dg[i - 1] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < kQlRun; ++t) {
                    const int i = i0 - t;
                    if (i < l) break;
                    const double f = sn * ei, b = cs * ei;
                    // r = sqrt(f^2 + g^2) and 1 / r from the hardware reciprocal square root
                    // with two Newton steps (a few ulp; the IEEE square root and division take
                    // a much longer dependent chain, and this recurrence runs on one lane)
                    const double s2 = fma(f, f, g * g);
                    if (s2 == 0.0) {
                        e[i + 1] = 0.0;
                        dg[i + 1] = di1 - p;
                        e[m] = 0.0;
                        early = true;
                        break;
                    }
                    const double rinv = rsqrt_nr(s2);
                    r = s2 * rinv;
                    e[i + 1] = r;
                    sn = f * rinv;
                    cs = g * rinv;
                    g = di1 - p;
                    r = (di - g) * sn + 2.0 * cs * b;
                    p = sn * r;
                    dg[i + 1] = g + p;
                    g = cs * r - b;
                    rc[cnt] = cs;
                    rs[cnt] = sn;
                    ++cnt;
                    di1 = di;
                    ei = en[t];
                    di = dn[t];
                }
            }
            if (!early) {
                dg[l] -= p;
                e[l] = g;
                e[m] = 0.0;
            }
            s_i0[buf] = m - 1;
            s_cnt[buf] = cnt;
            return;
        }
    };
    if (tid < 64) next_sweep(0);
    __syncthreads();
    for (int it = 0;; ++it) {
        const int cur = it & 1;
        if (s_done[cur]) break;
        if (tid < 64) {
            next_sweep(cur ^ 1);
        } else if (tid >= 64) {
            const int i0 = s_i0[cur], cnt = s_cnt[cur];
            const double* rc = rcl(cur);
            const double* rs = rsl(cur);
            // rotation t mixes columns i0 - t and i0 - t + 1; column i0 - t is read before any
            // rotation of the sweep writes it, so a chunk of reads goes out at once
            for (int row = tid - 64; row < d && cnt > 0; row += NT - 64) {
                double carry = Z[(int64_t)(i0 + 1) * d + row];
                for (int t0 = 0; t0 < cnt; t0 += kEigChunk) {
                    double zv[kEigChunk];
#pragma unroll
                    for (int u = 0; u < kEigChunk; ++u)
                        if (t0 + u < cnt) zv[u] = Z[(int64_t)(i0 - t0 - u) * d + row];
#pragma unroll
                    for (int u = 0; u < kEigChunk; ++u) {
                        const int t = t0 + u;
                        if (t < cnt) {
                            Z[(int64_t)(i0 - t + 1) * d + row] = rs[t] * zv[u] + rc[t] * carry;
                            carry = rc[t] * zv[u] - rs[t] * carry;
                        }
                    }
                }
                Z[(int64_t)(i0 - cnt + 1) * d + row] = carry;
            }
        }
        __syncthreads();
    }
    handover_barrier();                                 // rows of Z to the column owners
    for (int i = tid; i < d; i += NT) ev[B.eoff + i] = dg[i];
    }
    if (tid == 0 && zr == 1) atomicOr(&fail[blk], 2);   // Z column-major (QL path)
}

// sel: the sectors of the launch, one per work group
__global__ __launch_bounds__(kEigThreads) void k_heig(const DBlock* __restrict__ blks,
                                                      const int* __restrict__ sel,
                                                      dv2* __restrict__ A, double* __restrict__ Zb,
                                                      double* __restrict__ Sb,
                                                      double* __restrict__ ev, int* __restrict__ fail) {
    const int b = sel[blockIdx.x];
    heig<kEigThreads, kDensMaxDim, false>(blks[b], b, A, Zb, Sb, ev, fail);
}

// The same for sectors of at most kRegMaxDim states, with the matrix in registers in step 1.
__global__ __launch_bounds__(kEigThreadsR) void k_heig_r(const DBlock* __restrict__ blks,
                                                         const int* __restrict__ sel,
                                                         dv2* __restrict__ A,
                                                         double* __restrict__ Zb,
                                                         double* __restrict__ Sb,
                                                         double* __restrict__ ev,
                                                         int* __restrict__ fail) {
    const int b = sel[blockIdx.x];
    heig<kEigThreadsR, kRegMaxDim, true>(blks[b], b, A, Zb, Sb, ev, fail);
}

// Back-transformation Y = H_0 H_1 ... H_{d-2} Z of one sector's eigenvectors, BT reflectors
// at a time (back_bt(d): 8, or fewer above 256 states so that a block's reflectors fit in LDS),
// the block nearest the top padded with identity factors (zero reflector, tau = 0) so that
// every block has BT of them.  The product H_k1 ... H_k2 of a block is I - V T V^H (V the
// block's reflectors as columns, T upper triangular from the taus on the diagonal of A and the
// Gram matrix V^H V, T[r][c] = -tau_c sum_{r <= u < c} T[r][u] G[u][c], T[c][c] = tau_c).
//   k_back_t     the T of every block, in parallel (one work group per sector and block), into
//                Tb at blk.toff (block bi, from the bottom: bi BT^2 elements on, T[r][c] at
//                r + BT c);
//   k_heig_back  Y - V (T (V^H Y)) block after block, one work group per item of a host list
//                (a sector and its range of back_cols(d) columns of Y; larger sectors first, so
//                the longest work groups start first), the columns staying in LDS from the load
//                of Z (row-major, or
//                column-major when bit 1 of flags[blk] is set) to the store of Y (column-major).
//                The next block's reflectors and T are loaded into registers while the current
//                one is applied, and written to the other half of double LDS buffers, so a block
//                costs one barrier and no exposed global load.  kBackLanes (32) lanes per
//                column: lane q takes the rows i = q mod kBackLanes, and the lane group adds its
//                partial inner products by DPP rotations within each of its two rows of 16, then
//                a swizzle across them (the same bits in every lane).
static_assert(kBackLds / kDensMaxDim >= 1, "one column of the largest sector fits");
static_assert(kBackVs / 2 >= kDensMaxDim, "two reflectors of the largest sector fit");

// Reflector c of block bi (k = k1 + c), element i: 0 above the diagonal and for the padding,
// 1 on the subdiagonal, v below it (kept in A below the subdiagonal).
__device__ __forceinline__ dv2 back_v(const dv2* __restrict__ a, int d, int k, int i) {
    if (k < 0 || i <= k) return (dv2){0.0, 0.0};
    return i == k + 1 ? (dv2){1.0, 0.0} : a[(int64_t)k * d + i];
}

constexpr int kBackTThreads = 256;  // threads of k_back_t (8 per Gram entry, 28 entries)
template <int BT>
__device__ __forceinline__ void back_t(int d, int bi, const dv2* __restrict__ a,
                                       dv2* __restrict__ tg) {
    constexpr int NP = BT * (BT - 1) / 2, GL = 8;      // Gram pairs, lanes per pair
    __shared__ dv2 Vl[kBackVs], Gm[BT * BT], taus[BT];
    const int ln = threadIdx.x;
    const int k2 = d - 2 - bi * BT, k1 = k2 - BT + 1;
    for (int c = 0; c < BT; ++c)
        for (int i = ln; i < d; i += kBackTThreads) Vl[c * d + i] = back_v(a, d, k1 + c, i);
    if (ln < BT) taus[ln] = k1 + ln < 0 ? (dv2){0.0, 0.0} : a[(int64_t)(k1 + ln) * d + k1 + ln];
    __syncthreads();
    {
        // Gram entry (c1, c2), c1 < c2, by GL lanes (rows i = q mod GL), added by DPP moves
        const int p = ln / GL, q = ln % GL;
        dv2 acc = (dv2){0.0, 0.0};
        int c1 = 0, c2 = 1;
        if (p < NP) {
            int base = 0;                               // pairs with c2 = m start at m (m - 1) / 2
            while (base + c2 <= p) base += c2++;
            c1 = p - base;
            const int i0 = k1 + c2 + 1 > 0 ? k1 + c2 + 1 : 0;
            for (int i = i0 + q; i < d; i += GL) acc = cmac(acc, cconj(Vl[c1 * d + i]), Vl[c2 * d + i]);
        }
        // the 8 lanes of a pair are half a DPP row: lane ^ 1 and lane ^ 2 (quad permutations),
        // then lane 7 - i within the 8 (half-row mirror) give every lane the pair's sum
        static_assert(GL == 8, "a pair's lanes are half a DPP row");
        acc.x += dpp_shr<0xB1>(acc.x);
        acc.y += dpp_shr<0xB1>(acc.y);
        acc.x += dpp_shr<0x4E>(acc.x);
        acc.y += dpp_shr<0x4E>(acc.y);
        acc.x += dpp_shr<0x141>(acc.x);
        acc.y += dpp_shr<0x141>(acc.y);
        if (p < NP && q == 0) Gm[c1 + BT * c2] = acc;
    }
    __syncthreads();
    if (ln < BT) {
        const int r = ln;
        dv2 tr[BT];
#pragma unroll
        for (int c = 0; c < BT; ++c) {
            dv2 sum = (dv2){0.0, 0.0};
#pragma unroll
            for (int u = 0; u < c; ++u)
                if (u >= r) sum += cmul(tr[u], Gm[u + BT * c]);
            const dv2 tau = taus[c];
            tr[c] = r < c ? cmul((dv2){-tau.x, -tau.y}, sum) : (r == c ? tau : (dv2){0.0, 0.0});
        }
#pragma unroll
        for (int c = 0; c < BT; ++c) tg[(int64_t)bi * BT * BT + r + BT * c] = tr[c];
    }
}

__global__ __launch_bounds__(kBackTThreads) void k_back_t(const DBlock* __restrict__ blks,
                                               const dv2* __restrict__ A, dv2* __restrict__ Tb) {
    const DBlock B = blks[blockIdx.x];
    const int d = B.d, bi = blockIdx.y;
    if (bi >= back_nblocks(d)) return;
    const dv2* __restrict__ a = A + B.aoff;
    dv2* __restrict__ tg = Tb + B.toff;
    if (back_bt(d) == 8)
        back_t<8>(d, bi, a, tg);
    else if (back_bt(d) == 4)
        back_t<4>(d, bi, a, tg);
    else
        back_t<2>(d, bi, a, tg);
}

template <int BT>
__device__ __forceinline__ void back_blocks(int d, int nc, const dv2* __restrict__ a,
                                            const dv2* __restrict__ tg, dv2* __restrict__ Vs,
                                            dv2* __restrict__ Ys, dv2* __restrict__ Tt) {
    constexpr int NT = kBackThreads, L = kBackLanes;
    constexpr int PV = kBackVs / NT;                    // reflector elements a thread stages
    const int tid = threadIdx.x, q = tid % L, jl = tid / L;
    const int nb = back_nblocks(d);
    dv2 pv[PV], pt = (dv2){0.0, 0.0};
    auto fetch = [&](int bi) {                          // block bi into registers
        const int k1 = d - 2 - bi * BT - BT + 1;
#pragma unroll
        for (int u = 0; u < PV; ++u) {
            const int t = tid + u * NT, c = t / d, i = t - c * d;
            pv[u] = t < BT * d ? back_v(a, d, k1 + c, i) : (dv2){0.0, 0.0};
        }
        if (tid < BT * BT) pt = tg[(int64_t)bi * BT * BT + tid];
    };
    if (nb > 0) fetch(0);
    for (int bi = 0; bi < nb; ++bi) {
        dv2* __restrict__ V = Vs + (bi & 1) * kBackVs;
        dv2* __restrict__ T = Tt + (bi & 1) * BT * BT;
#pragma unroll
        for (int u = 0; u < PV; ++u)
            if (tid + u * NT < BT * d) V[tid + u * NT] = pv[u];
        if (tid < BT * BT) T[tid] = pt;
        __syncthreads();            // this block's buffers complete; the other buffers free
        if (bi + 1 < nb) fetch(bi + 1);
        const int k1 = d - 2 - bi * BT - BT + 1;
        if (jl < nc) {                                  // uniform over the lane group
            dv2* __restrict__ y = Ys + jl * d;
            const int i0 = k1 + 1 > 0 ? k1 + 1 : 0;     // rows above are not touched
            const int i1 = i0 + ((q - i0 % L) % L + L) % L;
            dv2 w[BT];
#pragma unroll
            for (int c = 0; c < BT; ++c) w[c] = (dv2){0.0, 0.0};
#pragma unroll 2
            for (int i = i1; i < d; i += L) {
                const dv2 yv = y[i];
#pragma unroll
                for (int c = 0; c < BT; ++c) w[c] = cmac(w[c], cconj(V[c * d + i]), yv);
            }
            static_assert(L == 16 || L == 32, "a lane group is one or two DPP rows");
            row_allsums(w);
            if constexpr (L == 32) {
#pragma unroll
                for (int c = 0; c < BT; ++c) {
                    w[c].x += swz16(w[c].x);
                    w[c].y += swz16(w[c].y);
                }
            }
            dv2 u[BT];
#pragma unroll
            for (int r = 0; r < BT; ++r) {
                u[r] = (dv2){0.0, 0.0};
#pragma unroll
                for (int c = r; c < BT; ++c) u[r] = cmac(u[r], T[r + BT * c], w[c]);
            }
#pragma unroll 2
            for (int i = i1; i < d; i += L) {
                dv2 yv = y[i];
#pragma unroll
                for (int c = 0; c < BT; ++c) yv = cmsc(yv, V[c * d + i], (dv2){u[c].x, -u[c].y});
                y[i] = yv;
            }
        }
    }
}

__global__ __launch_bounds__(kBackThreads) void k_heig_back(const DBlock* __restrict__ blks,
                                                            const DBackItem* __restrict__ items,
                                                            const dv2* __restrict__ A,
                                                            const dv2* __restrict__ Tb,
                                                            const double* __restrict__ Zb,
                                                            dv2* __restrict__ Yb,
                                                            const int* __restrict__ flags) {
    constexpr int NT = kBackThreads;
    const DBackItem it = items[blockIdx.x];
    const DBlock B = blks[it.blk];
    const int d = B.d, tid = threadIdx.x;
    const int cols = back_cols(d);
    const int jb = it.jb;
    const int nc = jb + cols < d ? cols : d - jb;       // columns jb .. jb + nc - 1
    const dv2* __restrict__ a = A + B.aoff;
    const dv2* __restrict__ tg = Tb + B.toff;
    const double* __restrict__ Z = Zb + B.aoff;
    dv2* __restrict__ Y = Yb + B.aoff;
    const bool colmajor = (flags[it.blk] & 2) != 0;
    const int64_t zr = colmajor ? 1 : d, zc = colmajor ? d : 1;
    __shared__ dv2 Vs[2 * kBackVs];                     // two blocks of reflectors, V[c d + i]
    __shared__ dv2 Ys[kBackLds];                        // Ys[jl d + i] = Y[i][jb + jl]
    __shared__ dv2 Tt[2 * 8 * 8];
    for (int jl = 0; jl < nc; ++jl)
        for (int i = tid; i < d; i += NT) Ys[jl * d + i] = (dv2){Z[i * zr + (jb + jl) * zc], 0.0};
    if (back_bt(d) == 8)
        back_blocks<8>(d, nc, a, tg, Vs, Ys, Tt);
    else if (back_bt(d) == 4)
        back_blocks<4>(d, nc, a, tg, Vs, Ys, Tt);
    else
        back_blocks<2>(d, nc, a, tg, Vs, Ys, Tt);
    __syncthreads();
    for (int jl = 0; jl < nc; ++jl)
        for (int i = tid; i < d; i += NT) Y[(int64_t)(jb + jl) * d + i] = Ys[jl * d + i];
}

// Global rank of eigenvalue g among all ntot (larger first, equal values by sector then index:
// the order of the flat array), in pieces: work group (x, y) counts, for its 256 eigenvalues,
// the values of chunk y (kRankChunk values through LDS) that rank before them, and adds the
// count to rank[g] (integer atomics: the sum does not depend on their order).  rank starts at
// zero (cleared by k_density).
constexpr int kRankChunk = 256;
__global__ __launch_bounds__(256) void k_rank(const double* __restrict__ ev, int ntot,
                                              int* __restrict__ rank) {
    __shared__ double sv[kRankChunk];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int h0 = blockIdx.y * kRankChunk;
    const int nh = ntot - h0 < kRankChunk ? ntot - h0 : kRankChunk;
    if (nh <= 0) return;
    for (int t = threadIdx.x; t < nh; t += blockDim.x) sv[t] = ev[h0 + t];
    __syncthreads();
    if (g >= ntot) return;
    const double x = ev[g];
    int r = 0;
    for (int t = 0; t < nh; ++t) {
        const double y = sv[t];
        r += (int)(y > x) | ((int)(y == x) & (int)(h0 + t < g));
    }
    if (r) atomicAdd(&rank[g], r);
}

constexpr int kFinishSplit = 8;     // work groups per sector of k_finish (the copy is shared)
// Per sector: eigenvalues in descending order (equal values by index) with their eigenvectors
// (two planes, column-major d x d at 2 blk.aoff in doubles: real parts, then imaginary parts),
// the number kept and the sums of all and of the kept eigenvalues.
__global__ __launch_bounds__(256) void k_finish(const DBlock* __restrict__ blks,
                                                const double* __restrict__ ev,
                                                const int* __restrict__ rank, int keep,
                                                const dv2* __restrict__ V,
                                                double* __restrict__ evals,
                                                double* __restrict__ evecs,
                                                int* __restrict__ nkept,
                                                double* __restrict__ sums) {
    const DBlock B = blks[blockIdx.x];
    const int d = B.d, tid = threadIdx.x;
    __shared__ double scratch[kVecThreads];
    __shared__ double se[kDensMaxDim];                  // the sector's eigenvalues
    __shared__ int src_of[kDensMaxDim];                 // output position r <- eigenvector i
    for (int i = tid; i < d; i += blockDim.x) se[i] = ev[B.eoff + i];
    __syncthreads();
    double all = 0.0, ksum = 0.0, kc = 0.0;
    const int ys = blockIdx.y, ny = gridDim.y;          // this work group's share of the copy
    for (int i = tid; i < d; i += blockDim.x) {
        const double x = se[i];
        int r = 0;
        for (int h = 0; h < d; ++h) r += (se[h] > x) || (se[h] == x && h < i);
        if (ys == 0) evals[B.eoff + r] = x;
        src_of[r] = i;
        all += x;
        if (rank[B.eoff + i] < keep) {
            ksum += x;
            kc += 1.0;
        }
    }
    __syncthreads();
    // V column-major (column i at V + aoff + i d): output column r (r = ys mod ny) is column
    // src_of[r] of V, copied along consecutive addresses
    {
        const dv2* __restrict__ src = V + B.aoff;
        double* __restrict__ dre = evecs + 2 * B.aoff;
        double* __restrict__ dim = dre + (int64_t)d * d;
        const int ncol = d > ys ? (d - ys + ny - 1) / ny : 0;
        const int nel = ncol * d;
#pragma unroll 4
        for (int o = tid; o < nel; o += blockDim.x) {
            const int rr = o / d, row = o - rr * d, r = ys + ny * rr;
            const dv2 z = src[(int64_t)src_of[r] * d + row];
            dre[(int64_t)r * d + row] = z.x;
            dim[(int64_t)r * d + row] = z.y;
        }
    }
    if (ys != 0) return;
    all = group_sum<kVecThreads>(all, scratch);
    ksum = group_sum<kVecThreads>(ksum, scratch);
    kc = group_sum<kVecThreads>(kc, scratch);
    if (tid == 0) {
        nkept[blockIdx.x] = (int)kc;
        sums[2 * blockIdx.x] = all;
        sums[2 * blockIdx.x + 1] = ksum;
    }
}

hipError_t launch_density(const DBlock* blks, int nblk, const int* sel, int nreg,
                          const DTile* tiles, int ntiles, const DensIn& in, int nv, int64_t n,
                          void* A, void* V, double* Z, double* S, void* Tb, int nbt, int* fail,
                          const DBackItem* back, int nback, double* ev,
                          int ntot, int keep, int* kept, double* evals, double* evecs, int* nkept,
                          double* sums, hipStream_t s) {
    hipLaunchKernelGGL(k_density, dim3(ntiles), dim3(64), 0, s, blks, tiles, in, nv, n,
                       static_cast<dv2*>(A), fail, nblk, kept, ntot);
    // sel: first the nreg sectors of the register-resident kernel, then the others
    if (nreg > 0)
        hipLaunchKernelGGL(k_heig_r, dim3(nreg), dim3(kEigThreadsR), 0, s, blks, sel,
                           static_cast<dv2*>(A), Z, S, ev, fail);
    if (nblk > nreg)
        hipLaunchKernelGGL(k_heig, dim3(nblk - nreg), dim3(kEigThreads), 0, s, blks, sel + nreg,
                           static_cast<dv2*>(A), Z, S, ev, fail);
    if (nbt > 0)
        hipLaunchKernelGGL(k_back_t, dim3(nblk, nbt), dim3(kBackTThreads), 0, s, blks,
                           static_cast<const dv2*>(A), static_cast<dv2*>(Tb));
    hipLaunchKernelGGL(k_heig_back, dim3(nback), dim3(kBackThreads), 0, s, blks, back,
                       static_cast<const dv2*>(A), static_cast<const dv2*>(Tb), Z,
                       static_cast<dv2*>(V), fail);
    hipLaunchKernelGGL(k_rank, dim3((ntot + 255) / 256, (ntot + kRankChunk - 1) / kRankChunk), dim3(256), 0,
                       s, ev, ntot, kept);
    hipLaunchKernelGGL(k_finish, dim3(nblk, kFinishSplit), dim3(256), 0, s, blks, ev, kept, keep,
                       static_cast<const dv2*>(V), evals, evecs, nkept, sums);
    return hipGetLastError();
}

}  // namespace dmrg
