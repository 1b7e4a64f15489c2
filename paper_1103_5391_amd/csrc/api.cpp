// C ABI of libdmrgtst (declared in include/dmrgtst.h): handle lifetime, device copies of the
// plan, and the launch sequences of H_sb.psi, the Krylov exponential (Sec. II.A, II.C) and
// time-step targeting (Sec. II.B, II.C).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/dmrgtst.h"
#include "internal.hpp"
#include "plan.hpp"
#include "tune_cache.hpp"

namespace dmrg {

hipError_t launch_stage1(int, int, const S1Block*, const Tile*, int, const ProbPtrs*, ProbPtrs,
                         hipStream_t);
hipError_t launch_stage2(int, int, const S2Block*, const Segment*, const Tile*, int,
                         const ProbPtrs*, ProbPtrs, hipStream_t);
hipError_t launch_stage2_mr(const S2Block*, const Segment*, const Tile*, int, const ProbPtrs*,
                            hipStream_t);
hipError_t launch_stage1_lds(int, const S1Block*, const LItem1*, int, const ProbPtrs*, ProbPtrs,
                             hipStream_t);
hipError_t launch_stage2_lds(int, const S2Block*, const Segment*, const LItem2*, int, const LRed*,
                             int, const ProbPtrs*, ProbPtrs, double*, hipStream_t);
hipError_t launch_stage1_x(const S1Block*, const LItem1*, int, const S2Block*, const XZero*, int,
                           const ProbPtrs*, ProbPtrs, hipStream_t);
hipError_t launch_stage2_x(const S2Block*, const XChunk*, const XItem2*, int, const ProbPtrs*,
                           ProbPtrs, hipStream_t);
hipError_t launch_stage1_k(const KXBlock*, const KPItem*, int, const KS1Block*, const KEdgeOut*,
                           const KTile*, int, const ProbPtrs*, ProbPtrs, hipStream_t);
hipError_t launch_stage2_k(const KS2Block*, const int64_t*, const KTile*, int, const ProbPtrs*,
                           ProbPtrs, hipStream_t);
hipError_t launch_start(const VecGroup&, const double*, const double* const*, int, int,
                        hipStream_t);
hipError_t launch_lanczos_iter(const VecGroup&, int, int, hipStream_t);
hipError_t launch_tridiag(const VecGroup&, const double*, int, int*, int, hipStream_t);
hipError_t launch_lowest(const VecGroup&, int*, int, hipStream_t);
hipError_t launch_count_nonfinite(const double*, int64_t, int*, hipStream_t);
hipError_t launch_density(const DBlock*, int, const int*, int, const DTile*, int, const DensIn&, int,
                          int64_t, void*, void*, double*, double*, void*, int, int*,
                          const DBackItem*, int, double*, int, int, int*, double*, double*, int*,
                          double*, hipStream_t);
hipError_t launch_combine(const VecGroup&, double* const*, double* const*, int, int, hipStream_t);
hipError_t launch_wft(const ZTile*, int, const ZPtrs&, const ZTile*, int, const ZPtrs&, int, int64_t,
                      hipStream_t);
hipError_t launch_zgemm(const ZTile*, int, const ZPtrs&, int, int, int, hipStream_t);
hipError_t launch_zero(double*, int64_t, hipStream_t);
hipError_t noalloc_scratch(double**);
hipError_t launch_local_mono(const SJob*, int, int64_t, const int*, const double*, const int*,
                             const double*, const double*, int64_t, double*, int64_t, hipStream_t);
hipError_t launch_zdot(const double*, const double*, int64_t, double*, int, hipStream_t);
constexpr int kDotBlocks = 256;     // partial sums of one inner product
int vec_blocks(int64_t n);
int red_blocks(int64_t n);

// Kernel families used until the autotuner or the caller chooses: register-tiled for both
// stages (the faster at the sizes measured so far).
constexpr int DMRG_GEMM_DEFAULT = 0;

// Device memory of one handle: a cap (DMRG_MAX_WORKSPACE bytes, read by dmrg_create; no cap
// without it) and the bytes its buffers hold.  The entry points make their handle's budget the
// current one for the calling thread; DevBuf allocations are charged to the current budget and
// refused (hipErrorOutOfMemory, reported as DMRG_ENOMEM) beyond its cap, before hipMalloc.
struct Budget {
    size_t cap = SIZE_MAX;
    size_t used = 0;
};
thread_local Budget* g_budget = nullptr;
struct BudgetScope {
    Budget* prev;
    explicit BudgetScope(Budget* b) : prev(g_budget) { g_budget = b; }
    ~BudgetScope() { g_budget = prev; }
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    Budget* owner = nullptr;      // budget the bytes are charged to
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        if (owner) owner->used -= bytes;
        p = nullptr;
        bytes = 0;
        owner = nullptr;
    }
    hipError_t alloc(size_t b) {
        release();
        if (b == 0) b = 8;
        Budget* bg = g_budget;
        if (bg && (b > bg->cap || bg->used > bg->cap - b)) return hipErrorOutOfMemory;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) {
            bytes = b;
            owner = bg;
            if (bg) bg->used += b;
        } else {
            p = nullptr;
        }
        return e;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Pinned host memory (hipHostMalloc), for results the host reads after a call.
struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~HostBuf() { release(); }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t b) {
        release();
        hipError_t e = hipHostMalloc(&p, b == 0 ? 8 : b, hipHostMallocDefault);
        if (e == hipSuccess)
            bytes = b;
        else
            p = nullptr;
        return e;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Device copies of the block-product work lists of one launch set (one handle, or the merged
// lists of a batch): stage descriptors per chunk depth (0: 16, 1: 32), tile lists of the
// register-tiled kernels (gemm.hip), tile lists of the LDS-tiled kernels (gemm_lds.hip) and
// their partial-tile workspace.
struct Lists {
    DevBuf dS1[2], dS2[2], dSeg[2], dT1, dT1n, dT2, dT2n, dL1, dL2[2], dLred[2], dPart;
    DevBuf dXch, dX2, dXz;    // LDS-staged family: chunk tables, stage-2 items, zeroed regions
    DevBuf dKX, dKP, dKS1, dKE, dKT1, dKS2, dKC, dKT2;   // K-split family
    int nt1 = 0, nt1n = 0, nt2 = 0, nt2n = 0, nl1 = 0, nl2[2] = {0, 0}, nred[2] = {0, 0};
    int nx2 = 0, nxz = 0;
    int nkp = 0, nkt1 = 0, nkt2 = 0;
    int variant = 0;    // DMRG_GEMM_* bits: which kernel family runs each stage
    // 4-RHS mode only: the owners' lists (each plan once), whose stage 2 runs all chains of a
    // tile in one work group (FP64, narrow tiles of both stages); nullptr elsewhere
    const Lists* mr = nullptr;
};

// Device copy of a host vector (synchronous on s).
template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    hipError_t e = b.alloc(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    e = hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// Uploads the work lists of one launch set; k indexes the chunk depth (0: 16, 1: 32).
hipError_t upload_lists(Lists& W, const std::vector<S1Block>* s1, const std::vector<S2Block>* s2,
                        const std::vector<Segment>* segs, const std::vector<Tile>& t1,
                        const std::vector<Tile>& t1n, const std::vector<Tile>& t2,
                        const std::vector<Tile>& t2n, const std::vector<LItem1>& l1,
                        const std::vector<LItem2>* l2, const std::vector<LRed>* lred,
                        const int* nslots, const std::vector<XChunk>& xch,
                        const std::vector<XItem2>& x2, const std::vector<XZero>& xz,
                        const KLists& kf, hipStream_t st) {
    hipError_t e = hipSuccess;
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = upload(W.dS1[k], s1[k], st);
        if (e == hipSuccess) e = upload(W.dS2[k], s2[k], st);
        if (e == hipSuccess) e = upload(W.dSeg[k], segs[k], st);
        if (e == hipSuccess) e = upload(W.dL2[k], l2[k], st);
        if (e == hipSuccess) e = upload(W.dLred[k], lred[k], st);
    }
    if (e == hipSuccess) e = upload(W.dT1, t1, st);
    if (e == hipSuccess) e = upload(W.dT1n, t1n, st);
    if (e == hipSuccess) e = upload(W.dT2, t2, st);
    if (e == hipSuccess) e = upload(W.dT2n, t2n, st);
    if (e == hipSuccess) e = upload(W.dL1, l1, st);
    if (e == hipSuccess) e = upload(W.dXch, xch, st);
    if (e == hipSuccess) e = upload(W.dX2, x2, st);
    if (e == hipSuccess) e = upload(W.dXz, xz, st);
    W.nx2 = (int)x2.size();
    W.nxz = (int)xz.size();
    if (e == hipSuccess) e = upload(W.dKX, kf.xblk, st);
    if (e == hipSuccess) e = upload(W.dKP, kf.pitems, st);
    if (e == hipSuccess) e = upload(W.dKS1, kf.s1, st);
    if (e == hipSuccess) e = upload(W.dKE, kf.eout, st);
    if (e == hipSuccess) e = upload(W.dKT1, kf.t1, st);
    if (e == hipSuccess) e = upload(W.dKS2, kf.s2, st);
    if (e == hipSuccess) e = upload(W.dKC, kf.ctab, st);
    if (e == hipSuccess) e = upload(W.dKT2, kf.t2, st);
    W.nkp = (int)kf.pitems.size();
    W.nkt1 = (int)kf.t1.size();
    W.nkt2 = (int)kf.t2.size();
    const int slots = std::max(nslots[0], nslots[1]);
    if (e == hipSuccess) e = W.dPart.alloc(sizeof(double) * (size_t)slots * kLTile * kLTile);
    W.nt1 = (int)t1.size();
    W.nt1n = (int)t1n.size();
    W.nt2 = (int)t2.size();
    W.nt2n = (int)t2n.size();
    W.nl1 = (int)l1.size();
    for (int k = 0; k < 2; ++k) {
        W.nl2[k] = (int)l2[k].size();
        W.nred[k] = (int)lred[k].size();
    }
    return e;
}

// One block-product stage (1 or 2) of one product for every problem of a launch set, with the
// kernel family the set's variant selects.
hipError_t run_stage(const Lists& W, int stage, int variant, int prec, const ProbPtrs* probs,
                     ProbPtrs single, hipStream_t s) {
    const int pk = prec >= DMRG_BF16X3 ? 1 : 0;
    // the K-split family: FP64, and only where the lists offer it (else register-tiled)
    if (variant & DMRG_GEMM_K) {
        if (prec == DMRG_FP64 && W.nkt2 > 0) {
            if (stage == 1)
                return launch_stage1_k(W.dKX.as<KXBlock>(), W.dKP.as<KPItem>(), W.nkp,
                                       W.dKS1.as<KS1Block>(), W.dKE.as<KEdgeOut>(),
                                       W.dKT1.as<KTile>(), W.nkt1, probs, single, s);
            return launch_stage2_k(W.dKS2.as<KS2Block>(), W.dKC.as<int64_t>(), W.dKT2.as<KTile>(),
                                   W.nkt2, probs, single, s);
        }
        variant = 0;
    }
    // the LDS-staged family: FP64, and only where the plan offers it (else register-tiled)
    if (variant & DMRG_GEMM_X) {
        if (prec == DMRG_FP64 && W.nx2 > 0) {
            if (stage == 1)
                return launch_stage1_x(W.dS1[0].as<S1Block>(), W.dL1.as<LItem1>(), W.nl1,
                                       W.dS2[0].as<S2Block>(), W.dXz.as<XZero>(), W.nxz, probs,
                                       single, s);
            return launch_stage2_x(W.dS2[0].as<S2Block>(), W.dXch.as<XChunk>(), W.dX2.as<XItem2>(),
                                   W.nx2, probs, single, s);
        }
        variant = 0;
    }
    if (stage == 1) {
        if (variant & DMRG_GEMM_STAGE1_LDS)
            return launch_stage1_lds(prec, W.dS1[pk].as<S1Block>(), W.dL1.as<LItem1>(), W.nl1,
                                     probs, single, s);
        if (variant & DMRG_GEMM_STAGE1_NARROW)
            return launch_stage1(prec, 1, W.dS1[pk].as<S1Block>(), W.dT1n.as<Tile>(), W.nt1n,
                                 probs, single, s);
        return launch_stage1(prec, 0, W.dS1[pk].as<S1Block>(), W.dT1.as<Tile>(), W.nt1, probs,
                             single, s);
    }
    if (variant & DMRG_GEMM_STAGE2_LDS)
        return launch_stage2_lds(prec, W.dS2[pk].as<S2Block>(), W.dSeg[pk].as<Segment>(),
                                 W.dL2[pk].as<LItem2>(), W.nl2[pk], W.dLred[pk].as<LRed>(),
                                 W.nred[pk], probs, single, W.dPart.as<double>(), s);
    if (variant & DMRG_GEMM_STAGE2_NARROW)
        return launch_stage2(prec, 1, W.dS2[pk].as<S2Block>(), W.dSeg[pk].as<Segment>(),
                             W.dT2n.as<Tile>(), W.nt2n, probs, single, s);
    return launch_stage2(prec, 0, W.dS2[pk].as<S2Block>(), W.dSeg[pk].as<Segment>(),
                         W.dT2.as<Tile>(), W.nt2, probs, single, s);
}

// Both block-product launches of one product.
hipError_t run_stages(const Lists& W, int prec, const ProbPtrs* probs, ProbPtrs single,
                      hipStream_t s) {
    const hipError_t e = run_stage(W, 1, W.variant, prec, probs, single, s);
    if (e != hipSuccess) return e;
    if (W.mr && probs && prec == DMRG_FP64 &&
        W.variant == (DMRG_GEMM_STAGE1_NARROW | DMRG_GEMM_STAGE2_NARROW)) {
        const Lists& M = *W.mr;
        return launch_stage2_mr(M.dS2[0].as<S2Block>(), M.dSeg[0].as<Segment>(),
                                M.dT2n.as<Tile>(), M.nt2n, probs, s);
    }
    return run_stage(W, 2, W.variant, prec, probs, single, s);
}

// Average milliseconds of `reps` back-to-back launches of one stage (after one untimed launch).
hipError_t time_stage(const Lists& W, int stage, int variant, int prec, const ProbPtrs* probs,
                      ProbPtrs single, hipStream_t s, int reps, double* ms) {
    hipEvent_t ev[2];
    hipError_t e = hipEventCreate(&ev[0]);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = run_stage(W, stage, variant, prec, probs, single, s);
    if (e == hipSuccess) e = hipEventRecord(ev[0], s);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
        e = run_stage(W, stage, variant, prec, probs, single, s);
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    *ms = (double)t / reps;
    return e;
}

// Autotuner of a launch set: each stage's kernel families timed in turn (stage 1 first, its
// output feeds stage 2), the fastest kept.  out: NULL or [s1 register, s1 LDS, s2 register,
// s2 LDS, s1 register narrow, s2 register narrow] ms.
hipError_t autotune_lists(Lists& W, int prec, const ProbPtrs* probs, ProbPtrs single,
                          hipStream_t s, int reps, double* out) {
    constexpr int kCand = 6;
    const int cand[kCand] = {0, DMRG_GEMM_STAGE1_LDS, 0, DMRG_GEMM_STAGE2_LDS,
                             DMRG_GEMM_STAGE1_NARROW, DMRG_GEMM_STAGE2_NARROW};
    const int stage[kCand] = {1, 1, 2, 2, 1, 2};
    double t[kCand];
    hipError_t e = hipSuccess;
    for (int i = 0; i < kCand && e == hipSuccess; ++i)
        e = time_stage(W, stage[i], cand[i], prec, probs, single, s, reps, &t[i]);
    if (e != hipSuccess) return e;
    int best[2] = {0, 2};   // fastest candidate of each stage (ties keep the register-tiled one)
    for (int i = 0; i < kCand; ++i)
        if (t[i] < t[best[stage[i] - 1]]) best[stage[i] - 1] = i;
    W.variant = cand[best[0]] | cand[best[1]];
    // the LDS-staged family runs both stages (its stage 1 zeroes what its stage 2 adds into):
    // timed as a pair, kept if the pair is faster
    double tx[2] = {-1.0, -1.0};
    if (prec == DMRG_FP64 && W.nx2 > 0) {
        for (int st = 1; st <= 2 && e == hipSuccess; ++st)
            e = time_stage(W, st, DMRG_GEMM_X, prec, probs, single, s, reps, &tx[st - 1]);
        if (e != hipSuccess) return e;
        if (tx[0] + tx[1] < t[best[0]] + t[best[1]]) W.variant = DMRG_GEMM_X;
    }
    // the K-split family likewise (its stage 1 writes the operand layout its stage 2 reads)
    double tk[2] = {-1.0, -1.0};
    if (prec == DMRG_FP64 && W.nkt2 > 0) {
        for (int st = 1; st <= 2 && e == hipSuccess; ++st)
            e = time_stage(W, st, DMRG_GEMM_K, prec, probs, single, s, reps, &tk[st - 1]);
        if (e != hipSuccess) return e;
        double cur = t[best[0]] + t[best[1]];
        if (W.variant == DMRG_GEMM_X) cur = tx[0] + tx[1];
        if (tk[0] + tk[1] < cur) W.variant = DMRG_GEMM_K;
    }
    if (out) {
        for (int i = 0; i < kCand; ++i) out[i] = t[i];
        out[kCand] = tx[0];
        out[kCand + 1] = tx[1];
        out[kCand + 2] = tk[0];
        out[kCand + 3] = tk[1];
    }
    return hipSuccess;
}

// Whether a dmrg_gemm variant is valid: known bits, at most one family per stage.
bool valid_variant(int32_t variant) {
    constexpr int32_t known = DMRG_GEMM_STAGE1_LDS | DMRG_GEMM_STAGE2_LDS |
                              DMRG_GEMM_STAGE1_NARROW | DMRG_GEMM_STAGE2_NARROW | DMRG_GEMM_X |
                              DMRG_GEMM_K;
    if (variant & ~known) return false;
    if ((variant & DMRG_GEMM_X) && variant != DMRG_GEMM_X) return false;
    if ((variant & DMRG_GEMM_K) && variant != DMRG_GEMM_K) return false;
    if ((variant & DMRG_GEMM_STAGE1_LDS) && (variant & DMRG_GEMM_STAGE1_NARROW)) return false;
    return !((variant & DMRG_GEMM_STAGE2_LDS) && (variant & DMRG_GEMM_STAGE2_NARROW));
}

// Device tables that run the Krylov passes of one handle, or of a batch of handles in common
// launches (one launch per pass for all problems), eagerly or as a captured HIP graph of the
// kdim Lanczos iterations.
struct Group {
    std::vector<dmrg_ctx*> hs;                 // member handles
    std::vector<int> rhs;                      // workspace of each member (chain index)
    Lists* lists = nullptr;                    // the handle's own, or the batch's merged lists
    DevBuf dVP, dBmap, dBmapR, dProbs, dIO;    // VecProb, block maps (streaming, reduction passes),
                                               // ProbPtrs[kMaxKrylov][nprob], IO
    VecGroup vg{};
    int prec = -1;                             // precision the tables were built for
    std::vector<uint64_t> gens;                // member workspace generations of the tables
    void** io_host = nullptr;                  // pinned staging of the per-call pointer table
    std::vector<const void*> io_last;          // content of the last upload
    hipEvent_t io_ev = nullptr;                // completion of the last upload
    bool use_graph = false;
    hipStream_t cap = nullptr;                 // private capture stream
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;  // captured iterations by (kdim, variant)

    void clear_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    ~Group() {
        clear_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        if (io_ev) (void)hipEventDestroy(io_ev);
        if (io_host) (void)hipHostFree(io_host);
    }
};

}  // namespace dmrg

using namespace dmrg;

namespace dmrg {

constexpr int kChains = 4;   // per-target chains of the 4-RHS mode (one per time-step target)

// Device workspace of one Krylov run: stage-1 intermediate, basis slots, work vector, partial
// sums, state.  A handle owns one per chain of the 4-RHS mode (the first also serves its
// single-chain calls); the others are allocated on first use.
struct Workspace {
    DevBuf dT;          // stage-1 intermediate
    DevBuf dV;          // Krylov basis slots
    DevBuf dW;          // matvec output / work vector
    DevBuf dPart;       // block partial sums
    DevBuf dState;      // KState
    int kcap = 0;       // basis slots allocated
    uint64_t gen = 0;   // bumped whenever a buffer is (re)allocated
};

}  // namespace dmrg

struct dmrg_batch_ctx {
    Lists lists;        // merged work lists of all members
    Lists mrl;          // 4-RHS mode: the owners' lists, each plan once (lists.mr)
    Group g;
    std::unique_ptr<dmrg_batch_ctx> chains;   // the 4-RHS mode: every member's four chains
};

struct dmrg_ctx {
    Budget budget;      // first member: destroyed after every buffer charged to it
    Plan plan;
    hipStream_t stream = nullptr;
    bool check_finite = false;          // check input vectors before a call (set_check_finite)
    DevBuf dCount;                      // non-finite count of the check
    DevBuf dKlog;                       // Lanczos vectors per step of one call
    int klog_cap = 0;
    int precision = DMRG_FP64;
    std::string last_error;
    // device copies of the plan's work lists, packed operators per arithmetic (built on
    // first use)
    Lists lists;
    DevBuf dA[4], dR[4];
    Workspace ws[kChains];
    Group self;         // tables of the handle's own Krylov runs
    // density matrix and truncation (built on first use): sectors, tiles, matrices, results
    // the call's results in one device area (per sector: the two sums, the number kept, the
    // eigen-decomposition flags), copied at once into pinned host memory
    DevBuf dDBlk, dDSel, dDTile, dDBack, dDA, dDV, dDZ, dDS, dDT, dDEv, dDKept, dDRes;
    HostBuf hDRes;
    int dens_ntiles = 0, dens_ntot = 0, dens_nreg = 0, dens_nbt = 0, dens_nback = 0;
    int64_t dens_nmat = 0;
    std::unique_ptr<dmrg_batch_ctx> chains;   // the handle's four chains of the 4-RHS mode
    // local operators (built on first use): raw operator blocks of both halves, the product
    // intermediate, the tile list and the inner-product partials
    DevBuf dOpS, dOpE, dLocT, dLocZ, dLocTiles, dLocPart, dLocJobs;
    std::vector<int64_t> opS_base, opE_base;
    // monomial operator blocks (at most one nonzero per row and column): per half the maps
    // (input index -> output index) and values, and per operator and source sector the offsets
    // of the map of the block (fwd) and of its transpose (bwd), -1 if the block is not monomial
    DevBuf dMonoMap[2], dMonoVal[2];
    std::vector<std::vector<int>> mono_fwd[2], mono_bwd[2];
    // the last planned call (terms and destination), whose device lists are reused when the
    // next call repeats it
    std::vector<dmrg_term> loc_terms;
    uint64_t loc_dst = 0;               // serial of the destination handle (0: none)
    uint64_t serial = 0;                // unique per handle in the process (never reused)
    std::vector<std::array<int, 5>> loc_launches;
    int64_t loc_tsize = 0;
};

// A planned move of the centre (wave-function transformation): tile lists of its two stages,
// the matrices W_r, and the intermediate.
struct dmrg_wft_ctx {
    dmrg_handle h = nullptr;
    DevBuf dTA, dTB, dW, dPhi;
    int nA = 0, nB = 0;
    int64_t nphi = 0;          // complex length of the intermediate of one vector
    int64_t n_new = 0;         // complex length of the new vector
    int phi_vecs = 0;          // vectors the intermediate is allocated for
    bool phi_zero = false;     // some intermediate rows are not written by stage A
    double flops_vec = 0.0;    // algorithmic flops per vector
};

namespace {

thread_local std::string g_create_error;

int fail(dmrg_handle h, int code, const std::string& msg) {
    if (h) h->last_error = msg;
    return code;
}

int hip_fail(dmrg_handle h, hipError_t e, const char* where) {
    if (e == hipErrorOutOfMemory)
        return fail(h, DMRG_ENOMEM, std::string(where) + ": device memory exhausted (or above the "
                                                         "handle's DMRG_MAX_WORKSPACE)");
    return fail(h, DMRG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, expr)                                     \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail((h), _e, #expr); \
    } while (0)


// Workspace r of a handle sized for kdim basis vectors (the stage-1 intermediate of workspace 0
// is allocated by dmrg_create; the padding rows of every intermediate are read (times zero
// factors) but never written, so intermediates start zeroed).
int ensure_workspace(dmrg_handle h, int kdim, int r = 0) {
    BudgetScope bs(&h->budget);
    Workspace& W = h->ws[r];
    if (W.kcap >= kdim + 1 && W.dW.p && W.dT.p) return DMRG_OK;
    const int64_t n2 = 2 * h->plan.n;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    ++W.gen;
    if (!W.dT.p) {
        const size_t bytes = sizeof(double) * (size_t)h->plan.T_size;
        HIP_TRY(h, W.dT.alloc(bytes));
        HIP_TRY(h, hipMemsetAsync(W.dT.p, 0, bytes, h->stream));
    }
    if (W.kcap < kdim + 1) {
        W.kcap = 0;                     // the old basis is released first, even on failure
        HIP_TRY(h, W.dV.alloc(sizeof(double) * (size_t)n2 * (kdim + 1)));
        W.kcap = kdim + 1;
    }
    if (!W.dW.p) HIP_TRY(h, W.dW.alloc(sizeof(double) * (size_t)n2));
    if (!W.dPart.p)
        HIP_TRY(h, W.dPart.alloc(sizeof(double) * (size_t)kDVals * kVecMaxBlocks *
                                 ((kMaxKrylov + kDSlots - 1) / kDSlots)));
    if (!W.dState.p) {
        HIP_TRY(h, W.dState.alloc(sizeof(KState)));
        HIP_TRY(h, hipMemsetAsync(W.dState.p, 0, sizeof(KState), h->stream));
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return DMRG_OK;
}

// Packed operators of one arithmetic on the device (built and cached on first use).
int ensure_operators(dmrg_handle h, int prec) {
    if (h->dA[prec].p && h->dR[prec].p) return DMRG_OK;
    BudgetScope bs(&h->budget);
    std::vector<uint8_t> A, R;
    try {
        pack_operators(h->plan, prec, A, R);
    } catch (const std::bad_alloc&) {
        return fail(h, DMRG_ENOMEM, "host memory for packed operators");
    }
    HIP_TRY(h, upload(h->dA[prec], A, h->stream));
    HIP_TRY(h, upload(h->dR[prec], R, h->stream));
    return DMRG_OK;
}

ProbPtrs make_ptrs(dmrg_handle h, int prec, const double* x, double* y, const int* skip,
                   int r = 0) {
    ProbPtrs pp;
    pp.x = x;
    pp.y = y;
    pp.T = h->ws[r].dT.p;
    pp.Lops = h->dA[prec].p;
    pp.Rops = h->dR[prec].p;
    pp.skip = skip;
    return pp;
}

// y = H_sb x for one caller vector.
int matvec_one(dmrg_handle h, const double* x, double* y) {
    const ProbPtrs pp = make_ptrs(h, h->precision, x, y, nullptr);
    HIP_TRY(h, run_stages(h->lists, h->precision, nullptr, pp, h->stream));
    return DMRG_OK;
}

// Makes the group's device tables match its members' workspaces for a run of size kdim.
int group_prepare(Group& g, int kdim) {
    dmrg_ctx* h0 = g.hs[0];
    const int prec = h0->precision;
    for (dmrg_ctx* h : g.hs)
        if (h->precision != prec) return fail(h0, DMRG_EINVAL, "batch members use different precisions");
    for (size_t i = 0; i < g.hs.size(); ++i) {
        dmrg_ctx* h = g.hs[i];
        const int rc = ensure_workspace(h, kdim, g.rhs[i]);
        if (rc) return h == h0 ? rc : fail(h0, rc, h->last_error);
    }
    bool stale = g.prec != prec || g.gens.size() != g.hs.size() || !g.dVP.p;
    for (size_t i = 0; !stale && i < g.hs.size(); ++i) stale = g.gens[i] != g.hs[i]->ws[g.rhs[i]].gen;
    if (!stale) return DMRG_OK;

    HIP_TRY(h0, hipStreamSynchronize(h0->stream));
    g.clear_graphs();
    const int np = (int)g.hs.size();
    std::vector<VecProb> vp(np);
    std::vector<int> bmap, bmapr;
    std::vector<ProbPtrs> pp((size_t)kMaxKrylov * np);
    int b0 = 0, b0r = 0;
    for (int i = 0; i < np; ++i) {
        dmrg_ctx* h = g.hs[i];
        const int r = g.rhs[i];
        Workspace& W = h->ws[r];
        const int64_t n = h->plan.n;
        double* V = W.dV.as<double>();
        KState* st = W.dState.as<KState>();
        const int nb = vec_blocks(n), nbr = red_blocks(n);
        vp[i] = VecProb{V, W.dW.as<double>(), W.dPart.as<double>(), st, n, 2 * n, nb, b0,
                        nbr, b0r};
        bmap.insert(bmap.end(), nb, i);
        bmapr.insert(bmapr.end(), nbr, i);
        b0 += nb;
        b0r += nbr;
        for (int j = 0; j < kMaxKrylov; ++j)
            // the products take slot j as it is (not yet normalised): no input scale
            pp[(size_t)j * np + i] = make_ptrs(h, prec, j < W.kcap ? V + (int64_t)j * 2 * n : nullptr,
                                               W.dW.as<double>(), &st->broken, r);
    }
    HIP_TRY(h0, upload(g.dVP, vp, h0->stream));
    if (np > 1) HIP_TRY(h0, upload(g.dBmap, bmap, h0->stream));
    if (np > 1) HIP_TRY(h0, upload(g.dBmapR, bmapr, h0->stream));
    HIP_TRY(h0, upload(g.dProbs, pp, h0->stream));
    g.vg = VecGroup{g.dVP.as<VecProb>(), np > 1 ? g.dBmap.as<int>() : nullptr,
                    np > 1 ? g.dBmapR.as<int>() : nullptr, np, b0, b0r, 4,
                    np == 1 ? vp[0] : VecProb{}};
    g.prec = prec;
    g.gens.resize(np);
    for (int i = 0; i < np; ++i) g.gens[i] = g.hs[i]->ws[g.rhs[i]].gen;
    return DMRG_OK;
}

// Both block-product launches of Lanczos iteration j for every problem of the group.
int group_matvec(Group& g, int j, hipStream_t s) {
    const ProbPtrs* probs = g.dProbs.as<ProbPtrs>() + (size_t)j * g.hs.size();
    HIP_TRY(g.hs[0], run_stages(*g.lists, g.prec, probs, ProbPtrs{}, s));
    return DMRG_OK;
}

// The kdim Lanczos iterations from the started slot 0, launched one by one.
int group_basis_eager(Group& g, int kdim, hipStream_t s) {
    for (int j = 0; j < kdim; ++j) {
        const int rc = group_matvec(g, j, s);
        if (rc) return rc;
        HIP_TRY(g.hs[0], launch_lanczos_iter(g.vg, j, kdim, s));
    }
    return DMRG_OK;
}

// The kdim Lanczos iterations: eager, or one launch of the graph captured for this kdim.
int group_basis(Group& g, int kdim, hipStream_t s) {
    if (!g.use_graph) return group_basis_eager(g, kdim, s);
    dmrg_ctx* h0 = g.hs[0];
    const std::pair<int, int> key(kdim, g.lists->variant);
    auto it = g.graphs.find(key);
    if (it == g.graphs.end()) {
        if (!g.cap) HIP_TRY(h0, hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking));
        HIP_TRY(h0, hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal));
        const int rc = group_basis_eager(g, kdim, g.cap);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(g.cap, &graph);
        if (rc || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc ? rc : hip_fail(h0, e, "hipStreamEndCapture");
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return hip_fail(h0, ei, "hipGraphInstantiate");
        it = g.graphs.emplace(key, ex).first;
    }
    HIP_TRY(h0, hipGraphLaunch(it->second, s));
    return DMRG_OK;
}

// Uploads the per-call pointer table of a batch: xt[nprob] then yst[nprob][kMaxTimes].
int group_io(Group& g, const std::vector<const void*>& io, hipStream_t s) {
    dmrg_ctx* h0 = g.hs[0];
    if (io == g.io_last) return DMRG_OK;
    const size_t bytes = io.size() * sizeof(void*);
    if (!g.io_host) HIP_TRY(h0, hipHostMalloc((void**)&g.io_host, bytes, hipHostMallocDefault));
    if (!g.io_ev) HIP_TRY(h0, hipEventCreateWithFlags(&g.io_ev, hipEventDisableTiming));
    if (!g.dIO.p) HIP_TRY(h0, g.dIO.alloc(bytes));
    HIP_TRY(h0, hipEventSynchronize(g.io_ev));   // the previous upload has left the staging
    std::memcpy(g.io_host, io.data(), bytes);
    HIP_TRY(h0, hipMemcpyAsync(g.dIO.p, g.io_host, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(h0, hipEventRecord(g.io_ev, s));
    g.io_last = io;
    return DMRG_OK;
}

void fill_info(const KState& st, dmrg_krylov_info* info) {
    info->converged = 1;
    info->k_eff = st.keff;
    info->k_eff_min = st.keff_min > kMaxKrylov ? st.keff : st.keff_min;
    info->beta0 = st.beta0_first;
    info->beta_last = st.keff > 0 ? st.beta[st.keff] : 0.0;
    info->err_est = st.err_est;
    info->breakdown = st.any_break;
}

// nsteps: entries of the per-step record to copy into info->k_eff_steps (if requested).
int read_info(dmrg_handle h, dmrg_krylov_info* info, int nsteps) {
    if (!info) return DMRG_OK;
    KState st;
    HIP_TRY(h, hipMemcpyAsync(&st, h->ws[0].dState.p, sizeof(KState), hipMemcpyDeviceToHost, h->stream));
    if (info->k_eff_steps && nsteps > 0)
        HIP_TRY(h, hipMemcpyAsync(info->k_eff_steps, h->dKlog.p, sizeof(int32_t) * (size_t)nsteps,
                                  hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    fill_info(st, info);
    if (st.nonfinite)
        return fail(h, DMRG_ENONFINITE, "a Krylov step started from a vector with a non-finite norm");
    if (st.exp_fail) return fail(h, DMRG_ENONFINITE, "Krylov exponential coefficients are not finite");
    return DMRG_OK;
}

// Device record of the Lanczos vectors per step, sized for nsteps (only when the caller asked
// for it through info->k_eff_steps); nullptr otherwise.
int klog_for(dmrg_handle h, const dmrg_krylov_info* info, int nsteps, int** out) {
    *out = nullptr;
    if (!info || !info->k_eff_steps || nsteps <= 0) return DMRG_OK;
    if (h->klog_cap < nsteps) {
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        h->klog_cap = 0;
        HIP_TRY(h, h->dKlog.alloc(sizeof(int32_t) * (size_t)nsteps));
        h->klog_cap = nsteps;
    }
    *out = h->dKlog.as<int>();
    return DMRG_OK;
}

// With checking on: DMRG_ENONFINITE if any of the count vectors (2n doubles each, device) holds
// a NaN or an infinity (the call waits for the stream); otherwise nothing.
int check_inputs(dmrg_handle h, const double* const* xs, int count) {
    if (!h->check_finite) return DMRG_OK;
    if (!h->dCount.p) HIP_TRY(h, h->dCount.alloc(sizeof(int)));
    HIP_TRY(h, hipMemsetAsync(h->dCount.p, 0, sizeof(int), h->stream));
    for (int i = 0; i < count; ++i)
        HIP_TRY(h, launch_count_nonfinite(xs[i], 2 * h->plan.n, h->dCount.as<int>(), h->stream));
    int bad = 0;
    HIP_TRY(h, hipMemcpyAsync(&bad, h->dCount.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (bad) return fail(h, DMRG_ENONFINITE, "input vector holds " + std::to_string(bad) +
                                                 " non-finite values");
    return DMRG_OK;
}

void tst_weights(double* weights) {
    if (!weights) return;
    const double W = 1.0 / 8.0;
    weights[0] = 2 * W;
    weights[1] = 2 * W;
    weights[2] = W;
    weights[3] = W;
    weights[4] = 2 * W;
}

// The launch set of the 4-RHS mode over `owners`: member 4 i + r is chain r of owners[i], with
// its own workspace; the work lists are the owners' plans, each repeated for its four chains, so
// every block-product launch carries all chains.  Built on first use.
int chains_set(std::unique_ptr<dmrg_batch_ctx>& cs, const std::vector<dmrg_ctx*>& owners) {
    if (cs) return DMRG_OK;
    dmrg_ctx* h0 = owners[0];
    std::unique_ptr<dmrg_batch_ctx> c(new (std::nothrow) dmrg_batch_ctx());
    if (!c) return fail(h0, DMRG_ENOMEM, "host memory for the chain tables");
    Group& g = c->g;
    g.lists = &c->lists;
    try {
        std::vector<const Plan*> plans;
        for (dmrg_ctx* h : owners)
            for (int r = 0; r < kChains; ++r) {
                g.hs.push_back(h);
                g.rhs.push_back(r);
                plans.push_back(&h->plan);
            }
        Merged M;
        merge_plans(plans, M);
        hipError_t e = upload_lists(c->lists, M.s1, M.s2, M.segs, M.tiles1, M.tiles1n,
                                    M.tiles2, M.tiles2n, M.l1, M.l2, M.lred, M.nslots,
                                    M.xch, M.x2, M.xz, M.kf, h0->stream);
        if (e == hipSuccess) {
            // the owners' lists for the shared-operator stage 2 (problem i = owner i)
            static_assert(kChains == kMultiRhs, "chain c of owner i is problem kChains i + c");
            std::vector<const Plan*> own;
            for (dmrg_ctx* h : owners) own.push_back(&h->plan);
            Merged O;
            merge_plans(own, O);
            e = upload_lists(c->mrl, O.s1, O.s2, O.segs, O.tiles1, O.tiles1n, O.tiles2,
                             O.tiles2n, O.l1, O.l2, O.lred, O.nslots, O.xch, O.x2, O.xz, O.kf,
                             h0->stream);
            c->lists.mr = &c->mrl;
        }
        if (e != hipSuccess)
            return fail(h0, e == hipErrorOutOfMemory ? DMRG_ENOMEM : DMRG_EHIP, hipGetErrorString(e));
    } catch (const std::bad_alloc&) {
        return fail(h0, DMRG_ENOMEM, "host memory for the chain tables");
    }
    cs = std::move(c);
    return DMRG_OK;
}

// One step of every chain of a 4-RHS launch set: targets[k] = exp(-i tau H) phi[k] (Krylov
// basis of kdim vectors from phi[k]; targets[k] may alias phi[k]).
int run_chains(dmrg_batch_ctx& cs, int variant, bool graph, const double* const* phi, double tau,
               int kdim, double* const* targets, dmrg_krylov_info* infos) {
    Group& g = cs.g;
    dmrg_ctx* h0 = g.hs[0];
    const int np = (int)g.hs.size();
    for (int i = 0; i < np; ++i)
        if (!phi[i] || !targets[i]) return fail(h0, DMRG_EINVAL, "NULL vector among the chains");
    cs.lists.variant = variant;
    g.use_graph = graph;
    int rc = group_prepare(g, kdim);
    if (rc) return rc;
    hipStream_t s = h0->stream;
    std::vector<const void*> io((size_t)np * (1 + kMaxTimes));
    for (int i = 0; i < np; ++i) {
        io[i] = phi[i];
        for (int x = 0; x < kMaxTimes; ++x) io[np + (size_t)i * kMaxTimes + x] = targets[i];
    }
    rc = group_io(g, io, s);
    if (rc) return rc;
    const double* const* xt = g.dIO.as<const double*>();
    double* const* yst = g.dIO.as<double*>() + np;
    HIP_TRY(h0, launch_start(g.vg, nullptr, xt, kdim, 1, s));
    rc = group_basis(g, kdim, s);
    if (rc) return rc;
    HIP_TRY(h0, launch_tridiag(g.vg, &tau, 1, nullptr, 0, s));
    HIP_TRY(h0, launch_combine(g.vg, nullptr, yst, 1, 0, s));
    if (!infos) return DMRG_OK;
    std::vector<KState> st(np);
    for (int i = 0; i < np; ++i)
        HIP_TRY(h0, hipMemcpyAsync(&st[i], g.hs[i]->ws[g.rhs[i]].dState.p, sizeof(KState),
                                   hipMemcpyDeviceToHost, s));
    HIP_TRY(h0, hipStreamSynchronize(s));
    for (int i = 0; i < np; ++i) {
        fill_info(st[i], &infos[i]);
        if (infos[i].k_eff_steps) infos[i].k_eff_steps[0] = st[i].keff;
    }
    for (int i = 0; i < np; ++i) {
        if (st[i].nonfinite)
            return fail(h0, DMRG_ENONFINITE, "a Krylov step started from a vector with a non-finite norm");
        if (st[i].exp_fail) return fail(h0, DMRG_ENONFINITE, "Krylov exponential coefficients are not finite");
    }
    return DMRG_OK;
}

// Validates a move description against the handle and builds the tile lists of both stages
// (host side of dmrg_wft_create).
int plan_wft(dmrg_handle h, const dmrg_wft_desc& D, std::vector<ZTile>& tA, std::vector<ZTile>& tB,
             std::vector<int64_t>& woff, dmrg_wft_ctx& w) {
    const Plan& P = h->plan;
    const int nb = (int)P.blocks.size();
    auto bad = [&](const char* why) { return fail(h, DMRG_EINVAL, std::string("wft: ") + why); };
    if (D.n_esub < 0 || D.nr < 0 || D.n_ssub < 0 || D.ns_new < 0 || D.ne_new < 0) return bad("negative count");
    if ((D.n_esub && !D.esub) || (D.nr && (!D.r_dim || !D.r_to_enew)) || (nb && !D.kept) ||
        (D.n_ssub && !D.ssub) || (D.ns_new && (!D.s_new_qn || !D.s_new_dim)) ||
        (D.ne_new && (!D.e_new_qn || !D.e_new_dim)))
        return bad("NULL table");
    for (int b = 0; b < nb; ++b)
        if (D.kept[b] < 0 || D.kept[b] > P.blocks[b].d) return bad("kept outside [0, d]");
    for (int r = 0; r < D.nr; ++r) {
        if (D.r_dim[r] < 0) return bad("negative R dimension");
        if (D.r_to_enew[r] < 0 || D.r_to_enew[r] >= D.ne_new) return bad("R sector maps outside E'");
        for (int r2 = 0; r2 < r; ++r2)
            if (D.r_to_enew[r2] == D.r_to_enew[r]) return bad("two R sectors map to one E' sector");
    }
    for (int i = 0; i < D.ns_new; ++i)
        if (D.s_new_dim[i] < 0) return bad("negative S' dimension");
    std::map<std::pair<int, int>, int> enew;
    for (int i = 0; i < D.ne_new; ++i) {
        if (D.e_new_dim[i] < 0) return bad("negative E' dimension");
        if (!enew.emplace(std::make_pair(D.e_new_qn[2 * i], D.e_new_qn[2 * i + 1]), i).second)
            return bad("repeated E' sector");
    }
    // W offsets (doubles): W_r is d_E'(r) x r_dim[r], two planes
    woff.assign(D.nr + 1, 0);
    for (int r = 0; r < D.nr; ++r)
        woff[r + 1] = woff[r] + 2 * (int64_t)D.e_new_dim[D.r_to_enew[r]] * D.r_dim[r];
    std::vector<int> r_of_enew(D.ne_new, -1);
    for (int r = 0; r < D.nr; ++r) r_of_enew[D.r_to_enew[r]] = r;
    // new layout: blocks (p', r') in S' order, r' the E' sector completing the target
    std::vector<int> col_of(D.ns_new, -1);
    std::vector<int64_t> new_off(D.ns_new, 0), phi_off(D.ns_new, -1);
    int64_t n_new = 0, nphi = 0;
    for (int i = 0; i < D.ns_new; ++i) {
        auto it = enew.find({P.target[0] - D.s_new_qn[2 * i], P.target[1] - D.s_new_qn[2 * i + 1]});
        if (it == enew.end()) continue;
        col_of[i] = it->second;
        new_off[i] = n_new;
        n_new += (int64_t)D.s_new_dim[i] * D.e_new_dim[it->second];
        const int r = r_of_enew[it->second];
        if (r >= 0) {
            phi_off[i] = nphi;
            nphi += (int64_t)D.s_new_dim[i] * D.r_dim[r];
        }
    }
    // sub-blocks of S': (b, a) -> (p', first row); rows covered at most once
    std::map<std::pair<int, int>, std::pair<int, int>> ssub;
    std::vector<std::vector<char>> used(D.ns_new);
    for (int i = 0; i < D.ns_new; ++i) used[i].assign(D.s_new_dim[i], 0);
    for (int i = 0; i < D.n_ssub; ++i) {
        const int* e = D.ssub + 4 * i;
        const int b = e[0], a = e[1], pp = e[2], roff = e[3];
        if (b < 0 || b >= nb || a < 0 || a > 3 || pp < 0 || pp >= D.ns_new || roff < 0 ||
            roff + D.kept[b] > D.s_new_dim[pp])
            return bad("S' sub-block outside its sector");
        if (!ssub.emplace(std::make_pair(b, a), std::make_pair(pp, roff)).second)
            return bad("repeated S' sub-block");
        for (int k = 0; k < D.kept[b]; ++k) {
            if (used[pp][roff + k]) return bad("S' rows covered twice");
            used[pp][roff + k] = 1;
        }
    }
    // stage A: one product per (kept block b, sub-block (a, r) of its E sector)
    std::vector<int64_t> uoff(nb + 1, 0);
    for (int b = 0; b < nb; ++b) uoff[b + 1] = uoff[b] + 2 * (int64_t)P.blocks[b].d * P.blocks[b].d;
    std::vector<int64_t> phi_rows(D.ns_new, 0);
    double flops = 0.0;
    auto tiles = [](std::vector<ZTile>& out, ZTile t) {
        for (int m0 = 0; m0 < std::max(t.M, 1); m0 += kZTile)
            for (int n0 = 0; n0 < t.N; n0 += kZTile) {
                t.m0 = m0;
                t.n0 = n0;
                out.push_back(t);
            }
    };
    for (int i = 0; i < D.n_esub; ++i) {
        const int* e = D.esub + 4 * i;
        const int q = e[0], a = e[1], r = e[2], coff = e[3];
        if (q < 0 || q >= P.E.nsec || a < 0 || a > 3 || r < 0 || r >= D.nr || coff < 0 ||
            coff + D.r_dim[r] > P.E.dim[q])
            return bad("E sub-block outside its sector");
        for (int b = 0; b < nb; ++b) {
            const PsiBlock& B = P.blocks[b];
            if (B.q != q || D.kept[b] == 0) continue;
            auto it = ssub.find({b, a});
            if (it == ssub.end()) return bad("kept sector without an S' sub-block for a site state");
            const int pp = it->second.first, roff = it->second.second;
            const int rr = D.r_to_enew[r];
            if (col_of[pp] != rr) return bad("quantum numbers do not add up to the target");
            // the site state moves the same quantum numbers on both sides
            if (P.E.nup[q] - D.e_new_qn[2 * rr] != D.s_new_qn[2 * pp] - P.S.nup[B.p] ||
                P.E.ndn[q] - D.e_new_qn[2 * rr + 1] != D.s_new_qn[2 * pp + 1] - P.S.ndn[B.p])
                return bad("site state with different quantum numbers on the two sides");
            ZTile t{};
            t.alpha = 1.0;
            t.M = D.kept[b];
            t.N = D.r_dim[r];
            t.K = B.d;
            t.amode = ZM_CT;
            t.aoff = uoff[b];
            t.aim = (int64_t)B.d * B.d;
            t.lda = B.d;
            t.bmode = ZM_COL;
            t.boff = B.off + (int64_t)coff * B.d;
            t.bim = P.n;
            t.ldb = B.d;
            t.coff = phi_off[pp] + roff;
            t.cim = 0;                    // set once the intermediate size is known
            t.ldc = D.s_new_dim[pp];
            if (t.N > 0 && t.M > 0) tiles(tA, t);
            flops += 8.0 * t.M * t.N * t.K;
            phi_rows[pp] += t.M;
        }
    }
    bool zero = false;
    for (int i = 0; i < D.ns_new; ++i)
        if (phi_off[i] >= 0 && D.r_dim[r_of_enew[col_of[i]]] > 0 && phi_rows[i] != D.s_new_dim[i]) zero = true;
    for (ZTile& t : tA) t.cim = nphi;
    // stage B: every new block, K = 0 where E' has no image of an R sector
    for (int i = 0; i < D.ns_new; ++i) {
        if (col_of[i] < 0) continue;
        const int rr = col_of[i], r = r_of_enew[rr];
        ZTile t{};
        t.alpha = 1.0;
        t.M = D.s_new_dim[i];
        t.N = D.e_new_dim[rr];
        t.K = r >= 0 ? D.r_dim[r] : 0;
        t.amode = ZM_COL;
        t.aoff = r >= 0 ? phi_off[i] : 0;
        t.aim = nphi;
        t.lda = std::max(1, D.s_new_dim[i]);
        t.bmode = ZM_CT;
        t.boff = r >= 0 ? woff[r] : 0;
        t.bim = r >= 0 ? (int64_t)D.e_new_dim[rr] * D.r_dim[r] : 0;
        t.ldb = std::max(1, D.e_new_dim[rr]);
        t.coff = new_off[i];
        t.cim = n_new;
        t.ldc = std::max(1, D.s_new_dim[i]);
        if (t.M > 0 && t.N > 0) tiles(tB, t);
        flops += 8.0 * t.M * t.N * t.K;
    }
    w.nphi = nphi;
    w.n_new = n_new;
    w.phi_zero = zero;
    w.flops_vec = flops;
    return DMRG_OK;
}

// Device copy of the raw operator blocks of both halves (first use of local operators).
int ensure_local_ops(dmrg_handle h) {
    if (h->dOpS.p && h->dOpE.p) return DMRG_OK;
    for (int side = 0; side < 2; ++side) {
        const HalfTable& T = side == 0 ? h->plan.S : h->plan.E;
        std::vector<double> all;
        std::vector<int64_t>& base = side == 0 ? h->opS_base : h->opE_base;
        base.clear();
        for (const HalfTable::Op& op : T.ops) {
            base.push_back((int64_t)all.size());
            all.insert(all.end(), op.data.begin(), op.data.end());
        }
        HIP_TRY(h, upload(side == 0 ? h->dOpS : h->dOpE, all, h->stream));
        // monomial blocks: maps of the block and of its transpose
        std::vector<int> maps;
        std::vector<double> vals;
        h->mono_fwd[side].assign(T.ops.size(), std::vector<int>(T.nsec, -1));
        h->mono_bwd[side].assign(T.ops.size(), std::vector<int>(T.nsec, -1));
        for (size_t o = 0; o < T.ops.size(); ++o) {
            const HalfTable::Op& op = T.ops[o];
            for (int p = 0; p < T.nsec; ++p) {
                if (op.boff[p] < 0) continue;
                const int q = T.find(T.nup[p] + op.dq[0], T.ndn[p] + op.dq[1]);
                const int rows = T.dim[q], cols = T.dim[p];
                const double* X = op.data.data() + op.boff[p];
                std::vector<int> fwd(cols, -1), bwd(rows, -1);
                std::vector<double> fv(cols, 0.0), bv(rows, 0.0);
                bool mono = true;
                for (int c = 0; c < cols && mono; ++c)
                    for (int r = 0; r < rows; ++r) {
                        const double v = X[(int64_t)c * rows + r];
                        if (v == 0.0) continue;
                        if (fwd[c] >= 0 || bwd[r] >= 0) {
                            mono = false;
                            break;
                        }
                        fwd[c] = r;
                        bwd[r] = c;
                        fv[c] = v;
                        bv[r] = v;
                    }
                if (!mono) continue;
                h->mono_fwd[side][o][p] = (int)maps.size();
                maps.insert(maps.end(), fwd.begin(), fwd.end());
                vals.insert(vals.end(), fv.begin(), fv.end());
                h->mono_bwd[side][o][p] = (int)maps.size();
                maps.insert(maps.end(), bwd.begin(), bwd.end());
                vals.insert(vals.end(), bv.begin(), bv.end());
            }
        }
        HIP_TRY(h, upload(h->dMonoMap[side], maps, h->stream));
        HIP_TRY(h, upload(h->dMonoVal[side], vals, h->stream));
    }
    return DMRG_OK;
}

// One factor of a local term on one half: the block that maps sector p (as source) and where
// it goes.  op < 0 is the identity.  Returns false if the factor has no block leaving p.
struct Factor {
    int dst;          // destination sector
    int mode;         // ZM_RCOL (op block), ZM_RT (transposed block), ZM_ID
    int64_t off;      // block offset (doubles) in the device copy
    int ld;           // leading dimension of the stored block
};

bool factor_of(const HalfTable& T, const std::vector<int64_t>& base, int op, int trans, int p,
               Factor& f) {
    if (op < 0) {
        f = Factor{p, ZM_ID, 0, 1};
        return true;
    }
    const HalfTable::Op& o = T.ops[op];
    if (!trans) {
        if (o.boff[p] < 0) return false;
        const int d = T.find(T.nup[p] + o.dq[0], T.ndn[p] + o.dq[1]);
        f = Factor{d, ZM_RCOL, base[op] + o.boff[p], T.dim[d]};
        return true;
    }
    // transposed: the block of op whose destination is p, from source p - dq
    const int src = T.find(T.nup[p] - o.dq[0], T.ndn[p] - o.dq[1]);
    if (src < 0 || o.boff[src] < 0) return false;
    f = Factor{src, ZM_RT, base[op] + o.boff[src], T.dim[p]};
    return true;
}

// Tile lists of y = sum_t coef_t (A_t P_S^f_t (x) B_t) x (src layout -> dst layout): per term,
// the right products T = X B^T (terms with an environment factor) then the left products
// y += alpha A T; launches[i] = (first tile, count, which product).
int plan_local(dmrg_handle hs, dmrg_handle hd, int nterm, const dmrg_term* terms,
               std::vector<ZTile>& tiles, std::vector<SJob>& jobs,
               std::vector<std::array<int, 5>>& launches, int64_t& tsize) {
    const Plan& S = hs->plan;
    const Plan& D = hd->plan;
    auto bad = [&](const std::string& why) { return fail(hs, DMRG_EINVAL, "local operator: " + why); };
    for (int side = 0; side < 2; ++side) {
        const HalfTable& a = side == 0 ? S.S : S.E;
        const HalfTable& b = side == 0 ? D.S : D.E;
        if (a.nup != b.nup || a.ndn != b.ndn || a.dim != b.dim) return bad("the handles have different halves");
    }
    tsize = 0;
    for (int t = 0; t < nterm; ++t) {
        const dmrg_term& tm = terms[t];
        if (tm.opS < -1 || tm.opS >= (int)S.S.ops.size() || tm.opE < -1 || tm.opE >= (int)S.E.ops.size())
            return bad("operator index out of range");
        if (!std::isfinite(tm.coef)) return fail(hs, DMRG_ENONFINITE, "local operator: coefficient is not finite");
        int dq[2] = {0, 0};
        if (tm.opS >= 0)
            for (int k = 0; k < 2; ++k) dq[k] += (tm.transS ? -1 : 1) * S.S.ops[tm.opS].dq[k];
        if (tm.opE >= 0)
            for (int k = 0; k < 2; ++k) dq[k] += (tm.transE ? -1 : 1) * S.E.ops[tm.opE].dq[k];
        if (S.target[0] + dq[0] != D.target[0] || S.target[1] + dq[1] != D.target[1])
            return bad("the term does not map the source sector to the destination sector");
        // monomial factors: every block this term uses maps one element to one element
        auto mono_of = [&](int side, int op, int trans, int p) -> int {
            if (op < 0) return -2;                              // identity
            const HalfTable& T = side == 0 ? S.S : S.E;
            if (!trans) return hs->mono_fwd[side][op][p];
            const int src = T.find(T.nup[p] - T.ops[op].dq[0], T.ndn[p] - T.ops[op].dq[1]);
            return src < 0 ? -1 : hs->mono_bwd[side][op][src];
        };
        bool mono = true;
        std::vector<SJob> tj;
        for (const PsiBlock& B : S.blocks) {
            Factor fa, fb;
            if (!factor_of(S.S, hs->opS_base, tm.opS, tm.transS, B.p, fa)) continue;
            if (!factor_of(S.E, hs->opE_base, tm.opE, tm.transE, B.q, fb)) continue;
            const int ob = fa.dst < (int)D.block_of_S.size() ? D.block_of_S[fa.dst] : -1;
            if (ob < 0 || D.blocks[ob].q != fb.dst) continue;
            const int ma = mono_of(0, tm.opS, tm.transS, B.p), mb = mono_of(1, tm.opE, tm.transE, B.q);
            if (ma == -1 || mb == -1) {
                mono = false;
                break;
            }
            const double sign = (tm.fermionic && ((S.S.nup[B.p] + S.S.ndn[B.p]) & 1)) ? -1.0 : 1.0;
            tj.push_back(SJob{B.off, D.blocks[ob].off, B.d, B.e, D.blocks[ob].d, ma < 0 ? -1 : ma,
                              mb < 0 ? -1 : mb, 0, tm.coef * sign});
        }
        if (mono) {
            if (!tj.empty()) {
                int64_t mx = 0;
                for (const SJob& j : tj) mx = std::max<int64_t>(mx, (int64_t)j.d * j.e);
                launches.push_back({(int)jobs.size(), (int)tj.size(), 3, (int)mx, 0});
                jobs.insert(jobs.end(), tj.begin(), tj.end());
            }
            continue;
        }
        std::vector<ZTile> right, left;
        int64_t toff = 0;
        for (const PsiBlock& B : S.blocks) {
            Factor fa, fb;
            if (!factor_of(S.S, hs->opS_base, tm.opS, tm.transS, B.p, fa)) continue;
            if (!factor_of(S.E, hs->opE_base, tm.opE, tm.transE, B.q, fb)) continue;
            const int ob = fa.dst < (int)D.block_of_S.size() ? D.block_of_S[fa.dst] : -1;
            if (ob < 0 || D.blocks[ob].q != fb.dst) continue;      // no such block in the target
            const PsiBlock& O = D.blocks[ob];
            const double sign = (tm.fermionic && ((S.S.nup[B.p] + S.S.ndn[B.p]) & 1)) ? -1.0 : 1.0;
            const int eo = S.E.dim[fb.dst];
            ZTile lt{};
            lt.alpha = tm.coef * sign;
            lt.acc = 1;
            lt.M = O.d;
            lt.N = eo;
            lt.K = B.d;
            lt.amode = fa.mode;
            lt.aoff = fa.off;
            lt.lda = fa.ld;
            lt.bmode = ZM_COL;
            lt.ldb = B.d;
            lt.coff = O.off;
            lt.cim = D.n;
            lt.ldc = O.d;
            if (fb.mode != ZM_ID) {
                ZTile rt{};
                rt.alpha = 1.0;
                rt.M = B.d;
                rt.N = eo;
                rt.K = B.e;
                rt.amode = ZM_COL;
                rt.aoff = B.off;
                rt.aim = S.n;
                rt.lda = B.d;
                rt.bmode = fb.mode == ZM_RCOL ? ZM_RT : ZM_RCOL;   // B^T of the stored block
                rt.boff = fb.off;
                rt.ldb = fb.ld;
                rt.coff = toff;
                rt.ldc = B.d;
                for (int m0 = 0; m0 < rt.M; m0 += kZTile)
                    for (int n0 = 0; n0 < rt.N; n0 += kZTile) {
                        rt.m0 = m0;
                        rt.n0 = n0;
                        right.push_back(rt);
                    }
                lt.boff = toff;
                lt.bim = -1;                  // the intermediate's plane offset, set below
                toff += (int64_t)B.d * eo;
            } else {
                lt.boff = B.off;
                lt.bim = S.n;
            }
            for (int m0 = 0; m0 < lt.M; m0 += kZTile)
                for (int n0 = 0; n0 < lt.N; n0 += kZTile) {
                    lt.m0 = m0;
                    lt.n0 = n0;
                    left.push_back(lt);
                }
        }
        for (ZTile& z : right) z.cim = toff;
        for (ZTile& z : left)
            if (z.bim < 0) z.bim = toff;
        tsize = std::max(tsize, toff);
        if (!right.empty()) {
            launches.push_back({(int)tiles.size(), (int)right.size(), 0, right[0].amode, right[0].bmode});
            tiles.insert(tiles.end(), right.begin(), right.end());
        }
        if (!left.empty()) {
            launches.push_back({(int)tiles.size(), (int)left.size(), tm.opE >= 0 ? 1 : 2, left[0].amode,
                                left[0].bmode});
            tiles.insert(tiles.end(), left.begin(), left.end());
        }
    }
    return DMRG_OK;
}

// y (dst layout) = sum of the terms applied to x (src layout); asynchronous.  launches[i] =
// (first tile, tiles, kind, A mode, B mode), kind 0 right products, 1 left products of the
// intermediate, 2 left products of x (the tiles of a launch share their operand modes), 3 a
// term with monomial factors (first job, jobs, kind, largest block's element count).
int run_local(dmrg_handle hs, dmrg_handle hd, int nterm, const dmrg_term* terms, const double* x,
              double* y) {
    int rc = ensure_local_ops(hs);
    if (rc) return rc;
    hipStream_t s = hs->stream;
    auto same = [](const dmrg_term& a, const dmrg_term& b) {
        return a.coef == b.coef && a.opS == b.opS && a.transS == b.transS && a.opE == b.opE &&
               a.transE == b.transE && a.fermionic == b.fermionic;
    };
    bool repeat = hs->loc_dst == hd->serial && (int)hs->loc_terms.size() == nterm;
    for (int t = 0; repeat && t < nterm; ++t) repeat = same(hs->loc_terms[t], terms[t]);
    if (!repeat) {
        std::vector<ZTile> tiles;
        std::vector<SJob> jobs;
        std::vector<std::array<int, 5>> launches;
        int64_t tsize = 0;
        hs->loc_dst = 0;
        rc = plan_local(hs, hd, nterm, terms, tiles, jobs, launches, tsize);
        if (rc) return rc;
        if ((int64_t)hs->dLocT.bytes < (int64_t)sizeof(double) * 2 * std::max<int64_t>(tsize, 1)) {
            HIP_TRY(hs, hipStreamSynchronize(s));
            HIP_TRY(hs, hs->dLocT.alloc(sizeof(double) * 2 * (size_t)std::max<int64_t>(tsize, 1)));
        }
        HIP_TRY(hs, upload(hs->dLocTiles, tiles, s));
        HIP_TRY(hs, upload(hs->dLocJobs, jobs, s));
        hs->loc_terms.assign(terms, terms + nterm);
        hs->loc_launches = launches;
        hs->loc_tsize = tsize;
        hs->loc_dst = hd->serial;
    }
    HIP_TRY(hs, launch_zero(y, 2 * hd->plan.n, s));
    for (const auto& L : hs->loc_launches) {
        if (L[2] == 3) {            // monomial factors: one element to one element
            HIP_TRY(hs, launch_local_mono(hs->dLocJobs.as<SJob>() + L[0], L[1], L[3], hs->dMonoMap[0].as<int>(),
                                          hs->dMonoVal[0].as<double>(), hs->dMonoMap[1].as<int>(),
                                          hs->dMonoVal[1].as<double>(), x, hs->plan.n, y, hd->plan.n, s));
            continue;
        }
        ZPtrs p{};
        if (L[2] == 0) {            // right products: x, environment blocks -> intermediate
            p.a[0] = x;
            p.b[0] = hs->dOpE.as<double>();
            p.c[0] = hs->dLocT.as<double>();
        } else {                    // left products: system blocks, intermediate or x -> y
            p.a[0] = hs->dOpS.as<double>();
            p.b[0] = L[2] == 1 ? hs->dLocT.as<double>() : x;
            p.c[0] = y;
        }
        HIP_TRY(hs, launch_zgemm(hs->dLocTiles.as<ZTile>() + L[0], L[1], p, 1, L[3], L[4], s));
    }
    return DMRG_OK;
}

int check_krylov_args(dmrg_handle h, double tau, int kdim) {
    if (kdim < 1 || kdim > kMaxKrylov) return fail(h, DMRG_EINVAL, "kdim outside [1, 64]");
    if (!std::isfinite(tau)) return fail(h, DMRG_ENONFINITE, "tau is not finite");
    return DMRG_OK;
}

}  // namespace

namespace {

// Whether the lists hold the work of every kernel family the variant names in arithmetic prec
// (a cache entry from another problem of the same key may name a family this one lacks).
bool runnable_variant(const Lists& W, int prec, int32_t v) {
    if (!valid_variant(v)) return false;
    if (v == DMRG_GEMM_X) return prec == DMRG_FP64 && W.nx2 > 0;
    if (v == DMRG_GEMM_K) return prec == DMRG_FP64 && W.nkt2 > 0;
    return true;
}

// Architecture name of the current device (gcnArchName up to its first ':').
hipError_t device_arch(std::string& arch) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return e;
    arch.assign(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return hipSuccess;
}

// Shared body of the cached autotuners: look key up, apply a runnable hit, else tune (tune()
// returns a status and fills the timings) and store.
template <class Tune>
int autotune_cached(dmrg_ctx* h, Lists& W, int prec, const std::string& key, const char* path,
                    double* out, int32_t* hit, Tune tune) {
    TuneEntry e;
    bool found = false;
    std::string err = tune_cache_find(path, key, e, found);
    if (!err.empty()) return fail(h, DMRG_EIO, err);
    if (found && runnable_variant(W, prec, e.variant)) {
        W.variant = e.variant;
        if (out) std::copy(e.ms, e.ms + kTuneTimes, out);
        if (hit) *hit = 1;
        return DMRG_OK;
    }
    const int rc = tune(e.ms);
    if (rc) return rc;
    e.key = key;
    e.variant = W.variant;
    if (out) std::copy(e.ms, e.ms + kTuneTimes, out);
    if (hit) *hit = 0;
    err = tune_cache_put(path, e);
    return err.empty() ? DMRG_OK : fail(h, DMRG_EIO, err);
}

}  // namespace

extern "C" {

int dmrg_create(const dmrg_problem* problem, void* stream, dmrg_handle* out) {
    if (!out) return DMRG_EINVAL;
    *out = nullptr;
    dmrg_ctx* h = new (std::nothrow) dmrg_ctx();
    if (!h) return DMRG_ENOMEM;
    static std::atomic<uint64_t> next_serial{1};
    h->serial = next_serial.fetch_add(1);
    try {
        g_create_error.clear();
        std::string err = build_plan(problem, h->plan);
        if (!err.empty()) {
            g_create_error = err;
            delete h;
            return DMRG_EINVAL;
        }
    } catch (const std::bad_alloc&) {
        delete h;
        return DMRG_ENOMEM;
    } catch (...) {
        delete h;
        return DMRG_EINVAL;
    }
    h->stream = static_cast<hipStream_t>(stream);
    h->self.hs.assign(1, h);
    h->self.rhs.assign(1, 0);
    if (const char* cap = std::getenv("DMRG_MAX_WORKSPACE")) {
        char* end = nullptr;
        const unsigned long long v = std::strtoull(cap, &end, 10);
        if (end == cap || *end != '\0') {
            g_create_error = "DMRG_MAX_WORKSPACE is not a byte count";
            delete h;
            return DMRG_EINVAL;
        }
        h->budget.cap = (size_t)v;
    }
    BudgetScope bs(&h->budget);
    const Plan& P = h->plan;
    hipError_t e = hipSuccess;
    h->self.lists = &h->lists;
    h->lists.variant = DMRG_GEMM_DEFAULT;
    {
        const std::vector<S1Block> s1[2] = {P.pk16.s1, P.pk32.s1};
        const std::vector<S2Block> s2[2] = {P.pk16.s2, P.pk32.s2};
        const std::vector<Segment> sg[2] = {P.pk16.segs, P.pk32.segs};
        const std::vector<LItem2> l2[2] = {P.pk16.l2, P.pk32.l2};
        const std::vector<LRed> lr[2] = {P.pk16.lred, P.pk32.lred};
        const int ns[2] = {P.pk16.nslots, P.pk32.nslots};
        e = upload_lists(h->lists, s1, s2, sg, P.tiles1, P.tiles1n, P.tiles2, P.tiles2n, P.l1, l2,
                         lr, ns, P.pk16.xch, P.pk16.x2, P.pk16.xz, P.kf, h->stream);
    }
    if (e == hipSuccess) e = h->ws[0].dT.alloc(sizeof(double) * (size_t)P.T_size);
    // the padding rows of the stage-1 workspace are read (times zero factors) but never
    // written: they must hold finite values, so the workspace starts zeroed
    if (e == hipSuccess)
        e = hipMemsetAsync(h->ws[0].dT.p, 0, sizeof(double) * (size_t)P.T_size, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        g_create_error = e == hipErrorOutOfMemory
                             ? "device memory exhausted (or above DMRG_MAX_WORKSPACE)"
                             : std::string(hipGetErrorString(e));
        delete h;
        return e == hipErrorOutOfMemory ? DMRG_ENOMEM : DMRG_EHIP;
    }
    if (const int rc = ensure_operators(h, DMRG_FP64)) {
        g_create_error = h->last_error;
        delete h;
        return rc;
    }
    {
        // set-up of the allocation-free entry point: the scratch array's address on this
        // device (once per device), resolved here so that later calls make no runtime query
        double* scr = nullptr;
        e = noalloc_scratch(&scr);
        if (e != hipSuccess) {
            g_create_error = std::string("device scratch of the allocation-free entry point: ") +
                             hipGetErrorString(e);
            delete h;
            return DMRG_EHIP;
        }
    }
    *out = h;
    return DMRG_OK;
}

void dmrg_destroy(dmrg_handle h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

int dmrg_psi_layout(dmrg_handle h, int64_t* n, int32_t* nblk, int64_t* off, int32_t* rows,
                    int32_t* cols, int32_t* secS, int32_t* secE) {
    if (!h) return DMRG_EINVAL;
    const Plan& P = h->plan;
    if (n) *n = P.n;
    if (nblk) *nblk = (int32_t)P.blocks.size();
    for (size_t b = 0; b < P.blocks.size(); ++b) {
        if (off) off[b] = P.blocks[b].off;
        if (rows) rows[b] = P.blocks[b].d;
        if (cols) cols[b] = P.blocks[b].e;
        if (secS) secS[b] = P.blocks[b].p;
        if (secE) secE[b] = P.blocks[b].q;
    }
    return DMRG_OK;
}

int dmrg_flops(dmrg_handle h, double* flops) {
    if (!h || !flops) return DMRG_EINVAL;
    *flops = h->plan.flops;
    return DMRG_OK;
}

int dmrg_plan_stats(const dmrg_problem* problem, int32_t kdim, dmrg_plan_info* out) {
    if (!problem || !out) return DMRG_EINVAL;
    if (kdim < 1 || kdim > kMaxKrylov) {
        g_create_error = "kdim outside [1, 64]";
        return DMRG_EINVAL;
    }
    try {
        g_create_error.clear();
        Plan P;
        const std::string err = build_plan(problem, P);
        if (!err.empty()) {
            g_create_error = err;
            return DMRG_EINVAL;
        }
        std::vector<uint8_t> A, R;
        pack_operators(P, DMRG_FP64, A, R);
        // the allocations of dmrg_create, in its order (a buffer of zero bytes takes 8)
        int64_t bytes = 0;
        auto add = [&](size_t b) { bytes += (int64_t)(b ? b : 8); };
        for (const Packing* pk : {&P.pk16, &P.pk32}) {
            add(pk->s1.size() * sizeof(S1Block));
            add(pk->s2.size() * sizeof(S2Block));
            add(pk->segs.size() * sizeof(Segment));
            add(pk->l2.size() * sizeof(LItem2));
            add(pk->lred.size() * sizeof(LRed));
        }
        add(P.tiles1.size() * sizeof(Tile));
        add(P.tiles1n.size() * sizeof(Tile));
        add(P.tiles2.size() * sizeof(Tile));
        add(P.tiles2n.size() * sizeof(Tile));
        add(P.l1.size() * sizeof(LItem1));
        add(P.pk16.xch.size() * sizeof(XChunk));
        add(P.pk16.x2.size() * sizeof(XItem2));
        add(P.pk16.xz.size() * sizeof(XZero));
        add(P.kf.xblk.size() * sizeof(KXBlock));
        add(P.kf.pitems.size() * sizeof(KPItem));
        add(P.kf.s1.size() * sizeof(KS1Block));
        add(P.kf.eout.size() * sizeof(KEdgeOut));
        add(P.kf.t1.size() * sizeof(KTile));
        add(P.kf.s2.size() * sizeof(KS2Block));
        add(P.kf.ctab.size() * sizeof(int64_t));
        add(P.kf.t2.size() * sizeof(KTile));
        add(sizeof(double) * (size_t)std::max(P.pk16.nslots, P.pk32.nslots) * kLTile * kLTile);
        add(sizeof(double) * (size_t)P.T_size);
        add(A.size());
        add(R.size());
        out->create_bytes = bytes;
        // the first Krylov call of kdim vectors: basis, work vector, partial sums, state, and
        // the handle's own group tables (descriptor, pointer table of every iteration)
        const size_t n2 = 2 * (size_t)P.n;
        out->krylov_bytes = (int64_t)(sizeof(double) * n2 * (size_t)(kdim + 1) + sizeof(double) * n2 +
                                      sizeof(double) * (size_t)kDVals * kVecMaxBlocks * kDMaxQ +
                                      sizeof(KState) + sizeof(VecProb) +
                                      sizeof(ProbPtrs) * (size_t)kMaxKrylov);
        out->n = P.n;
        out->nblk = (int32_t)P.blocks.size();
        out->flops = P.flops;
        out->flops_executed = P.flops_exec;
    } catch (const std::bad_alloc&) {
        return DMRG_ENOMEM;
    } catch (...) {
        return DMRG_EINVAL;
    }
    return DMRG_OK;
}

int dmrg_flops_executed(dmrg_handle h, double* flops) {
    if (!h || !flops) return DMRG_EINVAL;
    *flops = h->plan.flops_exec;
    return DMRG_OK;
}

int dmrg_set_precision(dmrg_handle h, int32_t precision) {
    if (!h) return DMRG_EINVAL;
    BudgetScope bs(&h->budget);
    if (precision < DMRG_FP64 || precision > DMRG_BF16X6)
        return fail(h, DMRG_EINVAL, "unknown precision");
    const int rc = ensure_operators(h, precision);
    if (rc) return rc;
    if (precision != h->precision) {
        // FP64 and the FP32-workspace arithmetics lay the stage-1 intermediate out with
        // different element sizes: padding positions of the new layout may hold bytes of the
        // old one, and they must be finite (they meet zero factors), so start from zeros again
        const size_t bytes = sizeof(double) * (size_t)h->plan.T_size;
        for (Workspace& W : h->ws)
            if (W.dT.p) HIP_TRY(h, hipMemsetAsync(W.dT.p, 0, bytes, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    h->precision = precision;
    return DMRG_OK;
}

int dmrg_set_stream(dmrg_handle h, void* stream) {
    if (!h) return DMRG_EINVAL;
    h->stream = static_cast<hipStream_t>(stream);
    return DMRG_OK;
}

int dmrg_matvec(dmrg_handle h, const double* x, double* y, int32_t nvec) {
    if (!h) return DMRG_EINVAL;
    if (nvec < 0 || (nvec > 0 && (!x || !y))) return fail(h, DMRG_EINVAL, "bad vectors");
    BudgetScope bs(&h->budget);
    const int64_t vs = 2 * h->plan.n;
    for (int v = 0; v < nvec; ++v) {
        const double* xv = x + v * vs;
        int rc = check_inputs(h, &xv, 1);
        if (rc) return rc;
    }
    for (int v = 0; v < nvec; ++v) {
        int rc = matvec_one(h, x + v * vs, y + v * vs);
        if (rc) return rc;
    }
    return DMRG_OK;
}

int dmrg_matvec_noalloc(dmrg_handle h, const double* x, double* y, int32_t nvec) {
    static_assert(kNoAllocScratchBytes == (size_t)DMRG_NOALLOC_SCRATCH_BYTES,
                  "scratch size of the header and of the library differ");
    if (!h) return DMRG_EINVAL;
    if (nvec < 0 || (nvec > 0 && (!x || !y))) return fail(h, DMRG_EINVAL, "bad vectors");
    if (nvec == 0) return DMRG_OK;
    // the part of the intermediate the handle's block-product family uses (the K-split
    // family pads it further)
    const int64_t tn = (h->lists.variant & DMRG_GEMM_K) && h->lists.nkt2 > 0
                           ? h->plan.kf.T_size
                           : h->plan.T_base;
    if ((size_t)tn * sizeof(double) > kNoAllocScratchBytes)
        return fail(h, DMRG_EINVAL, "the stage-1 intermediate takes " +
                                        std::to_string((size_t)tn * sizeof(double)) +
                                        " bytes, above the " +
                                        std::to_string(kNoAllocScratchBytes) +
                                        " bytes of the allocation-free scratch");
    double* T = nullptr;
    HIP_TRY(h, noalloc_scratch(&T));
    // the array holds whatever the last call on this GPU left: the intermediate's padding rows
    // meet zero factors and must be finite, so the used region starts from zeros (a fill
    // kernel, so that a captured call clears it on every replay)
    HIP_TRY(h, launch_zero(T, tn, h->stream));
    const int64_t vs = 2 * h->plan.n;
    for (int v = 0; v < nvec; ++v) {
        ProbPtrs pp = make_ptrs(h, h->precision, x + v * vs, y + v * vs, nullptr);
        pp.T = T;
        HIP_TRY(h, run_stages(h->lists, h->precision, nullptr, pp, h->stream));
    }
    return DMRG_OK;
}

int dmrg_krylov_expm(dmrg_handle h, const double* x, double* y, double tau, int32_t kdim,
                     int32_t nsteps, dmrg_krylov_info* info) {
    if (!h) return DMRG_EINVAL;
    if (!x || !y) return fail(h, DMRG_EINVAL, "NULL vector");
    if (nsteps < 0) return fail(h, DMRG_EINVAL, "negative nsteps");
    int rc = check_krylov_args(h, tau, kdim);
    if (rc) return rc;
    BudgetScope bs(&h->budget);
    rc = check_inputs(h, &x, 1);
    if (rc) return rc;
    if (nsteps == 0) {
        HIP_TRY(h, hipMemcpyAsync(y, x, sizeof(double) * 2 * h->plan.n, hipMemcpyDeviceToDevice,
                                  h->stream));
        if (info) {
            int32_t* steps = info->k_eff_steps;
            *info = dmrg_krylov_info{0, 0, 0.0, 0.0, 0.0, 0, 1, steps};
        }
        return DMRG_OK;
    }
    int* klog = nullptr;
    rc = klog_for(h, info, nsteps, &klog);
    if (rc) return rc;
    Group& g = h->self;
    rc = group_prepare(g, kdim);
    if (rc) return rc;
    HIP_TRY(h, launch_start(g.vg, x, nullptr, kdim, 1, h->stream));
    for (int s = 0; s < nsteps; ++s) {
        rc = group_basis(g, kdim, h->stream);
        if (rc) return rc;
        HIP_TRY(h, launch_tridiag(g.vg, &tau, 1, klog, s, h->stream));
        const bool last = s == nsteps - 1;
        double* out[1] = {y};
        HIP_TRY(h, launch_combine(g.vg, last ? out : nullptr, nullptr, 1, last ? 0 : 1, h->stream));
    }
    return read_info(h, info, nsteps);
}

int dmrg_tst_targets(dmrg_handle h, const double* phi, double tau, int32_t kdim, double* targets,
                     double* weights, dmrg_krylov_info* info) {
    if (!h) return DMRG_EINVAL;
    if (!phi || !targets) return fail(h, DMRG_EINVAL, "NULL vector");
    int rc = check_krylov_args(h, tau, kdim);
    if (rc) return rc;
    BudgetScope bs(&h->budget);
    rc = check_inputs(h, &phi, 1);
    if (rc) return rc;
    int* klog = nullptr;
    rc = klog_for(h, info, 1, &klog);
    if (rc) return rc;
    Group& g = h->self;
    rc = group_prepare(g, kdim);
    if (rc) return rc;
    const int64_t n = h->plan.n;
    HIP_TRY(h, launch_start(g.vg, phi, nullptr, kdim, 1, h->stream));
    rc = group_basis(g, kdim, h->stream);
    if (rc) return rc;
    const double times[4] = {0.0, tau / 3.0, 2.0 * tau / 3.0, tau};
    HIP_TRY(h, launch_tridiag(g.vg, times, 4, klog, 0, h->stream));
    double* out[4] = {targets, targets + 2 * n, targets + 4 * n, targets + 6 * n};
    HIP_TRY(h, launch_combine(g.vg, out, nullptr, 4, 0, h->stream));
    tst_weights(weights);
    return read_info(h, info, 1);
}

int dmrg_ground_state(dmrg_handle h, const double* x0, double* y, int32_t kdim,
                      int32_t max_restarts, double tol, double* energy, int32_t* restarts,
                      dmrg_krylov_info* info) {
    if (!h) return DMRG_EINVAL;
    if (!x0 || !y) return fail(h, DMRG_EINVAL, "NULL vector");
    if (max_restarts < 1) return fail(h, DMRG_EINVAL, "max_restarts < 1");
    if (!(tol >= 0.0)) return fail(h, DMRG_EINVAL, "tol must be a non-negative number");
    int rc = check_krylov_args(h, 0.0, kdim);
    if (rc) return rc;
    BudgetScope bs(&h->budget);
    rc = check_inputs(h, &x0, 1);
    if (rc) return rc;
    Group& g = h->self;
    rc = group_prepare(g, kdim);
    if (rc) return rc;
    HIP_TRY(h, launch_start(g.vg, x0, nullptr, kdim, 1, h->stream));
    KState st;
    int used = 0;
    bool converged = false;
    for (int r = 0; r < max_restarts; ++r) {
        rc = group_basis(g, kdim, h->stream);
        if (rc) return rc;
        HIP_TRY(h, launch_lowest(g.vg, nullptr, 0, h->stream));
        ++used;
        HIP_TRY(h, hipMemcpyAsync(&st, h->ws[0].dState.p, sizeof(KState), hipMemcpyDeviceToHost,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        if (st.nonfinite) return fail(h, DMRG_ENONFINITE, "start vector with a non-finite norm");
        if (st.exp_fail) return fail(h, DMRG_ENONFINITE, "ground-state eigenpair is not finite");
        if (info && info->k_eff_steps) info->k_eff_steps[r] = st.keff;
        // an invariant subspace (breakdown) makes the Ritz pair exact
        converged = st.err_est <= tol * std::max(1.0, std::fabs(st.eig)) || st.keff <= 0 ||
                    st.broken;
        const bool done = converged || r == max_restarts - 1;
        double* out[1] = {y};
        // converged (or out of restarts): the Ritz vector into y; else into slot 0, restart
        HIP_TRY(h, launch_combine(g.vg, done ? out : nullptr, nullptr, 1, done ? 0 : 1, h->stream));
        if (done) break;
    }
    if (energy) *energy = st.eig;
    if (restarts) *restarts = used;
    if (info) {
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        fill_info(st, info);
        info->converged = converged ? 1 : 0;
    }
    if (!converged) {
        h->last_error = "ground state: residual estimate above tol after max_restarts bases";
        return DMRG_WNOTCONV;
    }
    return DMRG_OK;
}

int dmrg_density_truncate(dmrg_handle h, const double* const* vecs, const double* weights,
                          int32_t nvec, int32_t keep, double* evals, double* evecs, int32_t* kept,
                          double* trunc_err) {
    if (!h) return DMRG_EINVAL;
    if (!vecs || !weights || !evals || !evecs || !kept) return fail(h, DMRG_EINVAL, "NULL pointer");
    if (nvec < 1 || nvec > kDensMaxVec) return fail(h, DMRG_EINVAL, "nvec outside [1, 16]");
    if (keep < 0) return fail(h, DMRG_EINVAL, "negative keep");
    BudgetScope bs(&h->budget);
    for (int l = 0; l < nvec; ++l) {
        if (!vecs[l]) return fail(h, DMRG_EINVAL, "NULL vector");
        if (!std::isfinite(weights[l])) return fail(h, DMRG_ENONFINITE, "weight is not finite");
    }
    const Plan& P = h->plan;
    const int nb = (int)P.blocks.size();
    hipStream_t s = h->stream;
    // result area: sums (2 nb doubles), numbers kept (nb ints), flags (nb ints)
    const size_t res_bytes = sizeof(double) * 2 * (size_t)nb + 2 * sizeof(int) * (size_t)nb;
    if (!h->dDBlk.p) {
        std::vector<DBlock> blks(nb);
        std::vector<DTile> tiles;
        std::vector<int> sel;
        int64_t aoff = 0, eoff = 0, toff = 0;
        for (int b = 0; b < nb; ++b) {
            const PsiBlock& pbk = P.blocks[b];
            if (pbk.d > kDensMaxDim) return fail(h, DMRG_EINVAL, "system sector larger than 1024");
            blks[b] = DBlock{pbk.d, pbk.e, pbk.off, aoff, eoff, toff};
            toff += (int64_t)back_nblocks(pbk.d) * back_bt(pbk.d) * back_bt(pbk.d);
            h->dens_nbt = std::max(h->dens_nbt, back_nblocks(pbk.d));
            if (pbk.d <= kDensRegMaxDim) sel.push_back(b);
            for (int i0 = 0; i0 < pbk.d; i0 += 16)       // tiles on and below the diagonal
                for (int j0 = 0; j0 <= i0; j0 += 16) tiles.push_back(DTile{b, i0, j0, 0});
            aoff += (int64_t)pbk.d * pbk.d;
            eoff += pbk.d;
        }
        h->dens_nreg = (int)sel.size();
        for (int b = 0; b < nb; ++b)
            if (P.blocks[b].d > kDensRegMaxDim) sel.push_back(b);
        // back-transformation work groups: every sector's column ranges, larger sectors first
        std::vector<int> order(nb);
        for (int b = 0; b < nb; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return P.blocks[x].d > P.blocks[y].d; });
        std::vector<DBackItem> back;
        for (int b : order)
            for (int jb = 0; jb < P.blocks[b].d; jb += back_cols(P.blocks[b].d))
                back.push_back(DBackItem{b, jb});
        h->dens_nback = (int)back.size();
        h->dens_ntiles = (int)tiles.size();
        h->dens_ntot = (int)eoff;
        h->dens_nmat = aoff;
        // the sector table goes last: it opens this block's gate, so a failed allocation
        // leaves every buffer to be allocated again by the next call
        HIP_TRY(h, upload(h->dDTile, tiles, s));
        HIP_TRY(h, upload(h->dDSel, sel, s));
        HIP_TRY(h, upload(h->dDBack, back, s));
        HIP_TRY(h, h->dDA.alloc(2 * sizeof(double) * (size_t)aoff));
        HIP_TRY(h, h->dDV.alloc(2 * sizeof(double) * (size_t)aoff));
        HIP_TRY(h, h->dDZ.alloc(sizeof(double) * (size_t)aoff));
        HIP_TRY(h, h->dDS.alloc(6 * sizeof(double) * (size_t)aoff));
        HIP_TRY(h, h->dDT.alloc(2 * sizeof(double) * (size_t)toff));
        HIP_TRY(h, h->dDEv.alloc(sizeof(double) * (size_t)eoff));
        HIP_TRY(h, h->dDKept.alloc(sizeof(int) * (size_t)eoff));
        HIP_TRY(h, h->dDRes.alloc(res_bytes));
        HIP_TRY(h, h->hDRes.alloc(res_bytes));
        HIP_TRY(h, upload(h->dDBlk, blks, s));
    }
    // per-call pointers and weights go by value in the launch
    DensIn in{};
    for (int l = 0; l < nvec; ++l) {
        in.v[l] = vecs[l];
        in.w[l] = weights[l];
    }
    double* d_sums = h->dDRes.as<double>();
    int* d_nk = reinterpret_cast<int*>(d_sums + 2 * (size_t)nb);
    int* d_flags = d_nk + nb;
    HIP_TRY(h, launch_density(h->dDBlk.as<DBlock>(), nb, h->dDSel.as<int>(), h->dens_nreg,
                              h->dDTile.as<DTile>(), h->dens_ntiles, in, nvec, P.n, h->dDA.p,
                              h->dDV.p, h->dDZ.as<double>(), h->dDS.as<double>(), h->dDT.p,
                              h->dens_nbt, d_flags, h->dDBack.as<DBackItem>(), h->dens_nback,
                              h->dDEv.as<double>(), h->dens_ntot, keep,
                              h->dDKept.as<int>(), evals, evecs, d_nk, d_sums, s));
    HIP_TRY(h, hipMemcpyAsync(h->hDRes.p, h->dDRes.p, res_bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    const double* sums = h->hDRes.as<double>();
    const int* nk = reinterpret_cast<const int*>(sums + 2 * (size_t)nb);
    const int* flags = nk + nb;
    for (int b = 0; b < nb; ++b)
        if (flags[b] & 1) return fail(h, DMRG_ENONFINITE, "density matrix: QL iteration did not converge");
    double all = 0.0, kept_sum = 0.0;
    for (int b = 0; b < nb; ++b) {
        kept[b] = nk[b];
        all += sums[2 * (size_t)b];
        kept_sum += sums[2 * (size_t)b + 1];
    }
    if (trunc_err) *trunc_err = all - kept_sum;
    return DMRG_OK;
}

int dmrg_wft_create(dmrg_handle h, const dmrg_wft_desc* desc, const double* const* W, dmrg_wft* out,
                    int64_t* n_new) {
    if (!out) return DMRG_EINVAL;
    *out = nullptr;
    if (!h) return DMRG_EINVAL;
    if (!desc) return fail(h, DMRG_EINVAL, "wft: NULL description");
    if (desc->nr > 0 && !W) return fail(h, DMRG_EINVAL, "wft: NULL W array");
    std::unique_ptr<dmrg_wft_ctx> w(new (std::nothrow) dmrg_wft_ctx());
    if (!w) return DMRG_ENOMEM;
    w->h = h;
    BudgetScope bs(&h->budget);
    std::vector<ZTile> tA, tB;
    std::vector<int64_t> woff;
    int rc = plan_wft(h, *desc, tA, tB, woff, *w);
    if (rc) return rc;
    for (int r = 0; r < desc->nr; ++r)
        if (woff[r + 1] > woff[r] && !W[r]) return fail(h, DMRG_EINVAL, "wft: NULL W matrix");
    hipStream_t s = h->stream;
    HIP_TRY(h, upload(w->dTA, tA, s));
    HIP_TRY(h, upload(w->dTB, tB, s));
    w->nA = (int)tA.size();
    w->nB = (int)tB.size();
    HIP_TRY(h, w->dW.alloc(sizeof(double) * (size_t)std::max<int64_t>(woff.back(), 1)));
    for (int r = 0; r < desc->nr; ++r)
        if (woff[r + 1] > woff[r])
            HIP_TRY(h, hipMemcpyAsync(w->dW.as<double>() + woff[r], W[r],
                                      sizeof(double) * (size_t)(woff[r + 1] - woff[r]),
                                      hipMemcpyDeviceToDevice, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    if (n_new) *n_new = w->n_new;
    *out = w.release();
    return DMRG_OK;
}

int dmrg_wft_apply(dmrg_wft w, const double* U, int32_t nvec, const double* const* x,
                   double* const* y, double* flops) {
    if (!w || !w->h) return DMRG_EINVAL;
    dmrg_handle h = w->h;
    if (nvec < 1 || nvec > kWftMaxVec) return fail(h, DMRG_EINVAL, "wft: nvec outside [1, 16]");
    if (!U || !x || !y) return fail(h, DMRG_EINVAL, "wft: NULL pointer");
    BudgetScope bs(&h->budget);
    for (int v = 0; v < nvec; ++v)
        if (!x[v] || !y[v]) return fail(h, DMRG_EINVAL, "wft: NULL vector");
    hipStream_t s = h->stream;
    if (w->phi_vecs < nvec) {
        HIP_TRY(h, hipStreamSynchronize(s));
        w->phi_vecs = 0;
        HIP_TRY(h, w->dPhi.alloc(sizeof(double) * 2 * (size_t)std::max<int64_t>(w->nphi, 1) * nvec));
        w->phi_vecs = nvec;
    }
    ZPtrs pA{}, pB{};
    double* phi = w->dPhi.as<double>();
    const int64_t stride = 2 * std::max<int64_t>(w->nphi, 1);
    for (int v = 0; v < nvec; ++v) {
        pA.a[v] = U;
        pA.b[v] = x[v];
        pA.c[v] = phi + v * stride;
        pB.a[v] = phi + v * stride;
        pB.b[v] = w->dW.as<double>();
        pB.c[v] = y[v];
    }
    HIP_TRY(h, launch_wft(w->dTA.as<ZTile>(), w->nA, pA, w->dTB.as<ZTile>(), w->nB, pB, nvec,
                          w->phi_zero ? stride : 0, s));
    if (flops) *flops = w->flops_vec * nvec;
    return DMRG_OK;
}

int dmrg_wft_destroy(dmrg_wft w) {
    if (!w) return DMRG_EINVAL;
    if (w->h) (void)hipStreamSynchronize(w->h->stream);
    delete w;
    return DMRG_OK;
}

int dmrg_apply_local(dmrg_handle src, dmrg_handle dst, int32_t nterm, const dmrg_term* terms,
                     const double* x, double* y) {
    if (!src || !dst) return DMRG_EINVAL;
    if (nterm < 1 || !terms || !x || !y) return fail(src, DMRG_EINVAL, "local operator: NULL or empty argument");
    if (x == y) return fail(src, DMRG_EINVAL, "local operator: y must not be x");
    BudgetScope bs(&src->budget);
    return run_local(src, dst, nterm, terms, x, y);
}

int dmrg_expect_local(dmrg_handle h, int32_t nterm, const dmrg_term* terms, const double* x,
                      double* re, double* im) {
    if (!h) return DMRG_EINVAL;
    if (nterm < 1 || !terms || !x) return fail(h, DMRG_EINVAL, "local operator: NULL or empty argument");
    BudgetScope bs(&h->budget);
    hipStream_t s = h->stream;
    if (!h->dLocZ.p) HIP_TRY(h, h->dLocZ.alloc(sizeof(double) * 2 * (size_t)h->plan.n));
    if (!h->dLocPart.p) HIP_TRY(h, h->dLocPart.alloc(sizeof(double) * 2 * kDotBlocks));
    int rc = run_local(h, h, nterm, terms, x, h->dLocZ.as<double>());
    if (rc) return rc;
    HIP_TRY(h, launch_zdot(x, h->dLocZ.as<double>(), h->plan.n, h->dLocPart.as<double>(), kDotBlocks, s));
    std::vector<double> part(2 * kDotBlocks);
    HIP_TRY(h, hipMemcpyAsync(part.data(), h->dLocPart.p, sizeof(double) * part.size(),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    double ar = 0.0, ai = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) {
        ar += part[2 * b];
        ai += part[2 * b + 1];
    }
    if (re) *re = ar;
    if (im) *im = ai;
    return DMRG_OK;
}

int dmrg_tst_chains(dmrg_handle h, const double* const* phi, double tau, int32_t kdim,
                    double* const* targets, double* weights, dmrg_krylov_info* infos) {
    if (!h) return DMRG_EINVAL;
    if (!phi || !targets) return fail(h, DMRG_EINVAL, "NULL pointer array");
    int rc = check_krylov_args(h, tau, kdim);
    if (rc) return rc;
    BudgetScope bs(&h->budget);
    for (int k = 0; k < kChains; ++k)
        if (!phi[k] || !targets[k]) return fail(h, DMRG_EINVAL, "NULL vector among the chains");
    rc = check_inputs(h, phi, kChains);
    if (rc) return rc;
    rc = chains_set(h->chains, std::vector<dmrg_ctx*>(1, h));
    if (rc) return rc;
    rc = run_chains(*h->chains, h->lists.variant, h->self.use_graph, phi, tau, kdim, targets, infos);
    if (rc) return rc;
    tst_weights(weights);
    return DMRG_OK;
}

int dmrg_set_check_finite(dmrg_handle h, int32_t enable) {
    if (!h) return DMRG_EINVAL;
    h->check_finite = enable != 0;
    return DMRG_OK;
}

int dmrg_set_graph(dmrg_handle h, int32_t enable) {
    if (!h) return DMRG_EINVAL;
    h->self.use_graph = enable != 0;
    return DMRG_OK;
}

int dmrg_batch_create(const dmrg_handle* handles, int32_t count, dmrg_batch* out) {
    if (!out) return DMRG_EINVAL;
    *out = nullptr;
    if (!handles || count <= 0) return DMRG_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!handles[i]) return DMRG_EINVAL;
    for (int i = 0; i < count; ++i)
        for (int k = 0; k < i; ++k)
            if (handles[k] == handles[i]) return fail(handles[0], DMRG_EINVAL, "handle repeated in a batch");
    dmrg_batch_ctx* b = new (std::nothrow) dmrg_batch_ctx();
    if (!b) return DMRG_ENOMEM;
    Group& g = b->g;
    g.hs.assign(handles, handles + count);
    g.rhs.assign(count, 0);
    g.lists = &b->lists;
    g.use_graph = true;
    dmrg_ctx* h0 = g.hs[0];
    BudgetScope bs(&h0->budget);
    try {
        std::vector<const Plan*> plans;
        for (dmrg_ctx* h : g.hs) plans.push_back(&h->plan);
        Merged M;
        merge_plans(plans, M);
        b->lists.variant = h0->lists.variant;
        const hipError_t e = upload_lists(b->lists, M.s1, M.s2, M.segs, M.tiles1, M.tiles1n, M.tiles2,
                                          M.tiles2n, M.l1, M.l2, M.lred, M.nslots, M.xch, M.x2,
                                          M.xz, M.kf, h0->stream);
        if (e != hipSuccess) {
            delete b;
            return fail(h0, e == hipErrorOutOfMemory ? DMRG_ENOMEM : DMRG_EHIP, hipGetErrorString(e));
        }
    } catch (const std::bad_alloc&) {
        delete b;
        return DMRG_ENOMEM;
    }
    *out = b;
    return DMRG_OK;
}

void dmrg_batch_destroy(dmrg_batch b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->g.hs[0]->stream);
    delete b;
}

int dmrg_batch_set_graph(dmrg_batch b, int32_t enable) {
    if (!b) return DMRG_EINVAL;
    b->g.use_graph = enable != 0;
    return DMRG_OK;
}

int dmrg_batch_tst_targets(dmrg_batch b, const double* const* phi, double tau, int32_t kdim,
                           double* const* targets, double* weights, dmrg_krylov_info* infos) {
    if (!b || !phi || !targets) return DMRG_EINVAL;
    Group& g = b->g;
    dmrg_ctx* h0 = g.hs[0];
    const int np = (int)g.hs.size();
    for (int i = 0; i < np; ++i)
        if (!phi[i] || !targets[i]) return fail(h0, DMRG_EINVAL, "NULL vector in a batch");
    int rc = check_krylov_args(h0, tau, kdim);
    if (rc) return rc;
    BudgetScope bs(&h0->budget);
    for (int i = 0; i < np; ++i) {
        rc = check_inputs(g.hs[i], &phi[i], 1);
        if (rc) return rc == DMRG_ENONFINITE ? fail(h0, rc, g.hs[i]->last_error) : rc;
    }
    rc = group_prepare(g, kdim);
    if (rc) return rc;
    hipStream_t s = h0->stream;
    std::vector<const void*> io((size_t)np * (1 + kMaxTimes));
    for (int i = 0; i < np; ++i) {
        const int64_t n = g.hs[i]->plan.n;
        io[i] = phi[i];
        for (int x = 0; x < kMaxTimes; ++x) io[np + (size_t)i * kMaxTimes + x] = targets[i] + 2 * n * x;
    }
    rc = group_io(g, io, s);
    if (rc) return rc;
    const double* const* xt = g.dIO.as<const double*>();
    double* const* yst = g.dIO.as<double*>() + np;
    HIP_TRY(h0, launch_start(g.vg, nullptr, xt, kdim, 1, s));
    rc = group_basis(g, kdim, s);
    if (rc) return rc;
    const double times[4] = {0.0, tau / 3.0, 2.0 * tau / 3.0, tau};
    HIP_TRY(h0, launch_tridiag(g.vg, times, 4, nullptr, 0, s));
    HIP_TRY(h0, launch_combine(g.vg, nullptr, yst, 4, 0, s));
    tst_weights(weights);
    if (!infos) return DMRG_OK;
    std::vector<KState> st(np);
    for (int i = 0; i < np; ++i)
        HIP_TRY(h0, hipMemcpyAsync(&st[i], g.hs[i]->ws[g.rhs[i]].dState.p, sizeof(KState),
                                   hipMemcpyDeviceToHost, s));
    HIP_TRY(h0, hipStreamSynchronize(s));
    for (int i = 0; i < np; ++i) {
        fill_info(st[i], &infos[i]);
        if (infos[i].k_eff_steps) infos[i].k_eff_steps[0] = st[i].keff;
    }
    for (int i = 0; i < np; ++i) {
        if (st[i].nonfinite)
            return fail(h0, DMRG_ENONFINITE, "a Krylov step started from a vector with a non-finite norm");
        if (st[i].exp_fail) return fail(h0, DMRG_ENONFINITE, "Krylov exponential coefficients are not finite");
    }
    return DMRG_OK;
}

int dmrg_batch_tst_chains(dmrg_batch b, const double* const* phi, double tau, int32_t kdim,
                          double* const* targets, double* weights, dmrg_krylov_info* infos) {
    if (!b || !phi || !targets) return DMRG_EINVAL;
    dmrg_ctx* h0 = b->g.hs[0];
    int rc = check_krylov_args(h0, tau, kdim);
    if (rc) return rc;
    BudgetScope bs(&h0->budget);
    rc = chains_set(b->chains, b->g.hs);
    if (rc) return rc;
    rc = run_chains(*b->chains, b->lists.variant, b->g.use_graph, phi, tau, kdim, targets, infos);
    if (rc) return rc;
    tst_weights(weights);
    return DMRG_OK;
}

int dmrg_profile_matvec(dmrg_handle h, const double* x, double* y, int32_t reps, double* out) {
    if (!h || !x || !y || !out || reps < 1) return DMRG_EINVAL;
    const int prec = h->precision;
    const ProbPtrs pp = make_ptrs(h, prec, x, y, nullptr);
    const int v = h->lists.variant;
    // stage 1 and stage 2 are idempotent (stage 1 rewrites the intermediate from x, stage 2
    // rewrites y from x and the intermediate): each is timed over back-to-back launches
    HIP_TRY(h, time_stage(h->lists, 1, v, prec, nullptr, pp, h->stream, reps, &out[0]));
    HIP_TRY(h, time_stage(h->lists, 2, v, prec, nullptr, pp, h->stream, reps, &out[1]));
    out[2] = h->plan.flops1;
    out[3] = h->plan.flops2;
    return DMRG_OK;
}

int dmrg_set_gemm(dmrg_handle h, int32_t variant) {
    if (!h) return DMRG_EINVAL;
    if (!valid_variant(variant))
        return fail(h, DMRG_EINVAL, "unknown kernel variant bits");
    h->lists.variant = variant;
    return DMRG_OK;
}

int dmrg_get_gemm(dmrg_handle h, int32_t* variant) {
    if (!h || !variant) return DMRG_EINVAL;
    *variant = h->lists.variant;
    return DMRG_OK;
}

int dmrg_autotune(dmrg_handle h, int32_t reps, double* out) {
    if (!h || reps < 1) return DMRG_EINVAL;
    BudgetScope bs(&h->budget);
    int rc = ensure_workspace(h, 1);
    if (rc) return rc;
    // timing inputs: basis slot 0 (zeroed) into the work vector
    const size_t bytes = sizeof(double) * 2 * (size_t)h->plan.n;
    HIP_TRY(h, hipMemsetAsync(h->ws[0].dV.p, 0, bytes, h->stream));
    const ProbPtrs pp = make_ptrs(h, h->precision, h->ws[0].dV.as<double>(), h->ws[0].dW.as<double>(),
                                  nullptr);
    HIP_TRY(h, autotune_lists(h->lists, h->precision, nullptr, pp, h->stream, reps, out));
    return DMRG_OK;
}

int dmrg_batch_set_gemm(dmrg_batch b, int32_t variant) {
    if (!b) return DMRG_EINVAL;
    if (!valid_variant(variant))
        return fail(b->g.hs[0], DMRG_EINVAL, "unknown kernel variant bits");
    b->lists.variant = variant;
    return DMRG_OK;
}

int dmrg_batch_autotune(dmrg_batch b, int32_t reps, double* out) {
    if (!b || reps < 1) return DMRG_EINVAL;
    Group& g = b->g;
    dmrg_ctx* h0 = g.hs[0];
    BudgetScope bs(&h0->budget);
    int rc = group_prepare(g, 1);
    if (rc) return rc;
    for (dmrg_ctx* h : g.hs)
        HIP_TRY(h0, hipMemsetAsync(h->ws[0].dV.p, 0, sizeof(double) * 2 * (size_t)h->plan.n, h0->stream));
    // row 0 of the product table: basis slot 0 into the work vector of every problem
    HIP_TRY(h0, autotune_lists(b->lists, g.prec, g.dProbs.as<ProbPtrs>(), ProbPtrs{}, h0->stream,
                               reps, out));
    return DMRG_OK;
}

int dmrg_autotune_cached(dmrg_handle h, const char* path, int32_t reps, double* out,
                         int32_t* hit) {
    if (!h || !path || reps < 1) return DMRG_EINVAL;
    try {
        std::string arch;
        HIP_TRY(h, device_arch(arch));
        const std::string key = tune_key({&h->plan}, h->precision, arch);
        return autotune_cached(h, h->lists, h->precision, key, path, out, hit,
                               [&](double* t) { return dmrg_autotune(h, reps, t); });
    } catch (const std::bad_alloc&) {
        return fail(h, DMRG_ENOMEM, "host allocation failed");
    }
}

int dmrg_batch_autotune_cached(dmrg_batch b, const char* path, int32_t reps, double* out,
                               int32_t* hit) {
    if (!b || !path || reps < 1) return DMRG_EINVAL;
    dmrg_ctx* h0 = b->g.hs[0];
    try {
        const int prec = h0->precision;
        std::vector<const Plan*> plans;
        for (dmrg_ctx* h : b->g.hs) {
            if (h->precision != prec)
                return fail(h0, DMRG_EINVAL, "batch members use different precisions");
            plans.push_back(&h->plan);
        }
        std::string arch;
        HIP_TRY(h0, device_arch(arch));
        const std::string key = tune_key(plans, prec, arch);
        return autotune_cached(h0, b->lists, prec, key, path, out, hit,
                               [&](double* t) { return dmrg_batch_autotune(b, reps, t); });
    } catch (const std::bad_alloc&) {
        return fail(h0, DMRG_ENOMEM, "host allocation failed");
    }
}

int dmrg_tune_key(const dmrg_problem* problem, int32_t precision, const char* arch, char* buf,
                  int64_t cap, int64_t* len) {
    if (!problem || !arch || !len || (buf && cap < 0)) return DMRG_EINVAL;
    if (precision < DMRG_FP64 || precision > DMRG_BF16X6) {
        g_create_error = "unknown precision";
        return DMRG_EINVAL;
    }
    try {
        g_create_error.clear();
        Plan P;
        const std::string err = build_plan(problem, P);
        if (!err.empty()) {
            g_create_error = err;
            return DMRG_EINVAL;
        }
        const std::string key = tune_key({&P}, precision, arch);
        *len = (int64_t)key.size();
        if (!buf) return DMRG_OK;
        if (cap <= (int64_t)key.size()) {
            g_create_error = "key buffer too short";
            return DMRG_EINVAL;
        }
        std::memcpy(buf, key.c_str(), key.size() + 1);
        return DMRG_OK;
    } catch (const std::bad_alloc&) {
        g_create_error = "host allocation failed";
        return DMRG_ENOMEM;
    }
}

int dmrg_tune_cache_lookup(const char* path, const char* key, int32_t* variant, double* ms,
                           int32_t* found) {
    if (!path || !key || !variant || !found) return DMRG_EINVAL;
    try {
        g_create_error.clear();
        TuneEntry e;
        bool f = false;
        const std::string err = tune_cache_find(path, key, e, f);
        if (!err.empty()) {
            g_create_error = err;
            return DMRG_EIO;
        }
        *found = f ? 1 : 0;
        if (f) {
            *variant = e.variant;
            if (ms) std::copy(e.ms, e.ms + kTuneTimes, ms);
        }
        return DMRG_OK;
    } catch (const std::bad_alloc&) {
        g_create_error = "host allocation failed";
        return DMRG_ENOMEM;
    }
}

int dmrg_tune_cache_store(const char* path, const char* key, int32_t variant, const double* ms) {
    if (!path || !key) return DMRG_EINVAL;
    if (!valid_variant(variant)) {
        g_create_error = "unknown kernel variant bits";
        return DMRG_EINVAL;
    }
    try {
        g_create_error.clear();
        TuneEntry e;
        e.key = key;
        e.variant = variant;
        for (int i = 0; i < kTuneTimes; ++i) e.ms[i] = ms ? ms[i] : -1.0;
        const std::string err = tune_cache_put(path, e);
        if (!err.empty()) {
            g_create_error = err;
            return DMRG_EIO;
        }
        return DMRG_OK;
    } catch (const std::bad_alloc&) {
        g_create_error = "host allocation failed";
        return DMRG_ENOMEM;
    }
}

const char* dmrg_strerror(int status) {
    switch (status) {
        case DMRG_OK: return "success";
        case DMRG_WNOTCONV: return "not converged (the last iterate is returned)";
        case DMRG_EINVAL: return "invalid argument";
        case DMRG_ENOMEM: return "out of memory";
        case DMRG_EHIP: return "HIP runtime error";
        case DMRG_ENONFINITE: return "non-finite value";
        case DMRG_ESTATE: return "invalid state";
        case DMRG_EIO: return "tuning cache file error";
        default: return "unknown status";
    }
}

const char* dmrg_last_error(dmrg_handle h) {
    return h ? h->last_error.c_str() : g_create_error.c_str();
}

}  // extern "C"
