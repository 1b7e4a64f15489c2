// C ABI of libdmrgtst (declared in include/dmrgtst.h): handle lifetime, device copies of the
// plan, and the launch sequences of H_sb.psi, the Krylov exponential (Sec. II.A, II.C) and
// time-step targeting (Sec. II.B, II.C).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dmrgtst.h"
#include "internal.hpp"
#include "plan.hpp"

namespace dmrg {

hipError_t launch_stage1(int, const S1Block*, const Tile*, int, const ProbPtrs*, ProbPtrs,
                         hipStream_t);
hipError_t launch_stage2(int, const S2Block*, const Segment*, const Tile*, int, const ProbPtrs*,
                         ProbPtrs, hipStream_t);
hipError_t launch_start(const double*, double*, int64_t, KState*, double*, int, int, hipStream_t);
hipError_t launch_lanczos_iter(double*, int64_t, double*, int64_t, int, int, KState*, double*,
                               hipStream_t);
hipError_t launch_tridiag(KState*, const double*, int, hipStream_t);
hipError_t launch_combine(const double*, int64_t, double* const*, int, int64_t, int, KState*,
                          double*, hipStream_t);

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t alloc(size_t b) {
        release();
        if (b == 0) b = 8;
        hipError_t e = hipMalloc(&p, b);
        if (e == hipSuccess) bytes = b;
        else p = nullptr;
        return e;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

}  // namespace dmrg

using namespace dmrg;

struct dmrg_ctx {
    Plan plan;
    hipStream_t stream = nullptr;
    int precision = DMRG_FP64;
    std::string last_error;
    // device copies of the plan: stage descriptors per chunk depth (0: 16, 1: 32), packed
    // operators per arithmetic (built on first use), tile lists
    DevBuf dS1[2], dS2[2], dSeg[2], dT1, dT2;
    DevBuf dA[3], dR[3];
    // workspace
    DevBuf dT;          // stage-1 intermediate
    DevBuf dV;          // Krylov basis slots
    DevBuf dW;          // matvec output / work vector
    DevBuf dPart;       // block partial sums
    DevBuf dState;      // KState
    int kcap = 0;       // basis slots allocated
};

struct dmrg_batch_ctx {
    std::vector<dmrg_handle> hs;
};

namespace {

thread_local std::string g_create_error;

int fail(dmrg_handle h, int code, const std::string& msg) {
    if (h) h->last_error = msg;
    return code;
}

int hip_fail(dmrg_handle h, hipError_t e, const char* where) {
    return fail(h, DMRG_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, expr)                                     \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail((h), _e, #expr); \
    } while (0)

template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    hipError_t e = b.alloc(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    if (v.empty()) return hipSuccess;
    e = hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

int ensure_workspace(dmrg_handle h, int kdim) {
    if (h->kcap >= kdim + 1 && h->dW.p) return DMRG_OK;
    const int64_t n2 = 2 * h->plan.n;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, h->dV.alloc(sizeof(double) * (size_t)n2 * (kdim + 1)));
    h->kcap = kdim + 1;
    if (!h->dW.p) HIP_TRY(h, h->dW.alloc(sizeof(double) * (size_t)n2));
    if (!h->dPart.p) HIP_TRY(h, h->dPart.alloc(sizeof(double) * 2 * kMaxKrylov * 1024));
    if (!h->dState.p) {
        HIP_TRY(h, h->dState.alloc(sizeof(KState)));
        HIP_TRY(h, hipMemsetAsync(h->dState.p, 0, sizeof(KState), h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    return DMRG_OK;
}

// Packed operators of one arithmetic on the device (built and cached on first use).
int ensure_operators(dmrg_handle h, int prec) {
    if (h->dA[prec].p) return DMRG_OK;
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

ProbPtrs make_ptrs(dmrg_handle h, const double* x, double* y, const double* xscale,
                   const int* skip) {
    ProbPtrs pp;
    pp.x = x;
    pp.y = y;
    pp.T = h->dT.p;
    pp.Lops = h->dA[h->precision].p;
    pp.Rops = h->dR[h->precision].p;
    pp.xscale = xscale;
    pp.skip = skip;
    return pp;
}

// y = H_sb x for one vector; x scaled by *xscale on load when non-null; skipped when *skip.
int matvec_one(dmrg_handle h, const double* x, double* y, const double* xscale, const int* skip) {
    const Plan& P = h->plan;
    const int prec = h->precision, pk = prec == DMRG_BF16X3 ? 1 : 0;
    const ProbPtrs pp = make_ptrs(h, x, y, xscale, skip);
    HIP_TRY(h, launch_stage1(prec, h->dS1[pk].as<S1Block>(), h->dT1.as<Tile>(),
                             (int)P.tiles1.size(), nullptr, pp, h->stream));
    HIP_TRY(h, launch_stage2(prec, h->dS2[pk].as<S2Block>(), h->dSeg[pk].as<Segment>(),
                             h->dT2.as<Tile>(), (int)P.tiles2.size(), nullptr, pp, h->stream));
    return DMRG_OK;
}

// One Lanczos basis of kdim vectors from the vector in slot 0 (already started).
int lanczos_basis(dmrg_handle h, int kdim) {
    const int64_t n = h->plan.n, vs = 2 * n;
    double* V = h->dV.as<double>();
    double* W = h->dW.as<double>();
    KState* st = h->dState.as<KState>();
    for (int j = 0; j < kdim; ++j) {
        int rc = matvec_one(h, V + (int64_t)j * vs, W, &st->scale[j], &st->broken);
        if (rc) return rc;
        HIP_TRY(h, launch_lanczos_iter(V, vs, W, n, j, kdim, st, h->dPart.as<double>(), h->stream));
    }
    return DMRG_OK;
}

int read_info(dmrg_handle h, dmrg_krylov_info* info) {
    if (!info) return DMRG_OK;
    KState st;
    HIP_TRY(h, hipMemcpyAsync(&st, h->dState.p, sizeof(KState), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    info->k_eff = st.keff;
    info->k_eff_min = st.keff_min > kMaxKrylov ? st.keff : st.keff_min;
    info->beta0 = st.beta0_first;
    info->beta_last = st.keff > 0 ? st.beta[st.keff] : 0.0;
    info->err_est = st.err_est;
    info->breakdown = st.any_break;
    if (st.eig_fail) return fail(h, DMRG_ENONFINITE, "tridiagonal eigensolver did not converge");
    return DMRG_OK;
}

}  // namespace

extern "C" {

int dmrg_create(const dmrg_problem* problem, void* stream, dmrg_handle* out) {
    if (!out) return DMRG_EINVAL;
    *out = nullptr;
    dmrg_ctx* h = new (std::nothrow) dmrg_ctx();
    if (!h) return DMRG_ENOMEM;
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
    const Plan& P = h->plan;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload(h->dS1[0], P.pk16.s1, h->stream);
    if (e == hipSuccess) e = upload(h->dS2[0], P.pk16.s2, h->stream);
    if (e == hipSuccess) e = upload(h->dSeg[0], P.pk16.segs, h->stream);
    if (e == hipSuccess) e = upload(h->dS1[1], P.pk32.s1, h->stream);
    if (e == hipSuccess) e = upload(h->dS2[1], P.pk32.s2, h->stream);
    if (e == hipSuccess) e = upload(h->dSeg[1], P.pk32.segs, h->stream);
    if (e == hipSuccess) e = upload(h->dT1, P.tiles1, h->stream);
    if (e == hipSuccess) e = upload(h->dT2, P.tiles2, h->stream);
    if (e == hipSuccess) e = h->dT.alloc(sizeof(double) * (size_t)P.T_size);
    // the padding rows of the stage-1 workspace are read (times zero factors) but never
    // written: they must hold finite values, so the workspace starts zeroed
    if (e == hipSuccess) e = hipMemsetAsync(h->dT.p, 0, sizeof(double) * (size_t)P.T_size, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return e == hipErrorOutOfMemory ? DMRG_ENOMEM : DMRG_EHIP;
    }
    if (ensure_operators(h, DMRG_FP64) != DMRG_OK) {
        g_create_error = h->last_error;
        delete h;
        return DMRG_ENOMEM;
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

int dmrg_set_precision(dmrg_handle h, int32_t precision) {
    if (!h) return DMRG_EINVAL;
    if (precision != DMRG_FP64 && precision != DMRG_FP32 && precision != DMRG_BF16X3)
        return fail(h, DMRG_EINVAL, "unknown precision");
    const int rc = ensure_operators(h, precision);
    if (rc) return rc;
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
    const int64_t vs = 2 * h->plan.n;
    for (int v = 0; v < nvec; ++v) {
        int rc = matvec_one(h, x + v * vs, y + v * vs, nullptr, nullptr);
        if (rc) return rc;
    }
    return DMRG_OK;
}

int dmrg_krylov_expm(dmrg_handle h, const double* x, double* y, double tau, int32_t kdim,
                     int32_t nsteps, dmrg_krylov_info* info) {
    if (!h) return DMRG_EINVAL;
    if (!x || !y) return fail(h, DMRG_EINVAL, "NULL vector");
    if (kdim < 1 || kdim > kMaxKrylov) return fail(h, DMRG_EINVAL, "kdim outside [1, 64]");
    if (nsteps < 0) return fail(h, DMRG_EINVAL, "negative nsteps");
    if (!std::isfinite(tau)) return fail(h, DMRG_ENONFINITE, "tau is not finite");
    int rc = ensure_workspace(h, kdim);
    if (rc) return rc;
    const int64_t n = h->plan.n;
    double* V = h->dV.as<double>();
    KState* st = h->dState.as<KState>();
    double* part = h->dPart.as<double>();
    if (nsteps == 0) {
        HIP_TRY(h, hipMemcpyAsync(y, x, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, h->stream));
        if (info) *info = dmrg_krylov_info{0, 0, 0.0, 0.0, 0.0, 0};
        return DMRG_OK;
    }
    HIP_TRY(h, launch_start(x, V, n, st, part, kdim, 1, h->stream));
    for (int s = 0; s < nsteps; ++s) {
        rc = lanczos_basis(h, kdim);
        if (rc) return rc;
        HIP_TRY(h, launch_tridiag(st, &tau, 1, h->stream));
        const bool last = s == nsteps - 1;
        double* out[1] = {last ? y : V};
        HIP_TRY(h, launch_combine(V, 2 * n, out, 1, n, last ? 0 : 1, st, part, h->stream));
    }
    return read_info(h, info);
}

int dmrg_tst_targets(dmrg_handle h, const double* phi, double tau, int32_t kdim, double* targets,
                     double* weights, dmrg_krylov_info* info) {
    if (!h) return DMRG_EINVAL;
    if (!phi || !targets) return fail(h, DMRG_EINVAL, "NULL vector");
    if (kdim < 1 || kdim > kMaxKrylov) return fail(h, DMRG_EINVAL, "kdim outside [1, 64]");
    if (!std::isfinite(tau)) return fail(h, DMRG_ENONFINITE, "tau is not finite");
    int rc = ensure_workspace(h, kdim);
    if (rc) return rc;
    const int64_t n = h->plan.n;
    double* V = h->dV.as<double>();
    KState* st = h->dState.as<KState>();
    double* part = h->dPart.as<double>();
    HIP_TRY(h, launch_start(phi, V, n, st, part, kdim, 1, h->stream));
    rc = lanczos_basis(h, kdim);
    if (rc) return rc;
    const double times[4] = {0.0, tau / 3.0, 2.0 * tau / 3.0, tau};
    HIP_TRY(h, launch_tridiag(st, times, 4, h->stream));
    double* out[4] = {targets, targets + 2 * n, targets + 4 * n, targets + 6 * n};
    HIP_TRY(h, launch_combine(V, 2 * n, out, 4, n, 0, st, part, h->stream));
    if (weights) {
        const double W = 1.0 / 8.0;
        weights[0] = 2 * W;
        weights[1] = 2 * W;
        weights[2] = W;
        weights[3] = W;
        weights[4] = 2 * W;
    }
    return read_info(h, info);
}

int dmrg_batch_create(const dmrg_handle* handles, int32_t count, dmrg_batch* out) {
    if (!out) return DMRG_EINVAL;
    *out = nullptr;
    if (!handles || count <= 0) return DMRG_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!handles[i]) return DMRG_EINVAL;
    dmrg_batch_ctx* b = new (std::nothrow) dmrg_batch_ctx();
    if (!b) return DMRG_ENOMEM;
    b->hs.assign(handles, handles + count);
    *out = b;
    return DMRG_OK;
}

void dmrg_batch_destroy(dmrg_batch b) { delete b; }

int dmrg_batch_tst_targets(dmrg_batch b, const double* const* phi, double tau, int32_t kdim,
                           double* const* targets, double* weights, dmrg_krylov_info* infos) {
    if (!b || !phi || !targets) return DMRG_EINVAL;
    for (size_t i = 0; i < b->hs.size(); ++i) {
        int rc = dmrg_tst_targets(b->hs[i], phi[i], tau, kdim, targets[i], weights,
                                  infos ? infos + i : nullptr);
        if (rc) return rc;
    }
    return DMRG_OK;
}

int dmrg_profile_matvec(dmrg_handle h, const double* x, double* y, int32_t reps, double* out) {
    if (!h || !x || !y || !out || reps < 1) return DMRG_EINVAL;
    const Plan& P = h->plan;
    const int prec = h->precision, pk = prec == DMRG_BF16X3 ? 1 : 0;
    const ProbPtrs pp = make_ptrs(h, x, y, nullptr, nullptr);
    hipEvent_t ev[3];
    for (auto& e : ev) HIP_TRY(h, hipEventCreate(&e));
    double t1 = 0.0, t2 = 0.0;
    for (int r = 0; r < reps; ++r) {
        HIP_TRY(h, hipEventRecord(ev[0], h->stream));
        HIP_TRY(h, launch_stage1(prec, h->dS1[pk].as<S1Block>(), h->dT1.as<Tile>(),
                                 (int)P.tiles1.size(), nullptr, pp, h->stream));
        HIP_TRY(h, hipEventRecord(ev[1], h->stream));
        HIP_TRY(h, launch_stage2(prec, h->dS2[pk].as<S2Block>(), h->dSeg[pk].as<Segment>(),
                                 h->dT2.as<Tile>(), (int)P.tiles2.size(), nullptr, pp, h->stream));
        HIP_TRY(h, hipEventRecord(ev[2], h->stream));
        HIP_TRY(h, hipEventSynchronize(ev[2]));
        float a = 0.f, b = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&a, ev[0], ev[1]));
        HIP_TRY(h, hipEventElapsedTime(&b, ev[1], ev[2]));
        t1 += a;
        t2 += b;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    out[0] = t1 / reps;
    out[1] = t2 / reps;
    out[2] = P.flops1;
    out[3] = P.flops2;
    return DMRG_OK;
}

const char* dmrg_strerror(int status) {
    switch (status) {
        case DMRG_OK: return "success";
        case DMRG_EINVAL: return "invalid argument";
        case DMRG_ENOMEM: return "out of memory";
        case DMRG_EHIP: return "HIP runtime error";
        case DMRG_ENONFINITE: return "non-finite value";
        case DMRG_ESTATE: return "invalid state";
        default: return "unknown status";
    }
}

const char* dmrg_last_error(dmrg_handle h) {
    return h ? h->last_error.c_str() : g_create_error.c_str();
}

}  // extern "C"
