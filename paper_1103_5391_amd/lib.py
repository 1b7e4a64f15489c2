"""ctypes binding of libdmrgtst.so (C ABI in include/dmrgtst.h).

Argument marshalling only: every step of H_sb.psi, the Krylov exponential and time-step
targeting runs in the library's HIP kernels.  Vectors are torch tensors (float64, contiguous,
on the GPU) used as plain device buffers; streams are torch's current HIP stream.  There is no
CPU fallback: loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# DMRG_LIB selects another build of the same library (the sanitized host build in the tests)
LIB_PATH = os.environ.get("DMRG_LIB") or os.path.join(HERE, "libdmrgtst.so")

DMRG_FP64, DMRG_FP32, DMRG_BF16X3, DMRG_BF16X6 = 0, 1, 2, 3
DMRG_GEMM_STAGE1_LDS, DMRG_GEMM_STAGE2_LDS = 1, 2
DMRG_GEMM_STAGE1_NARROW, DMRG_GEMM_STAGE2_NARROW = 4, 8
DMRG_GEMM_X = 16
DMRG_GEMM_K = 32
STATUS = {0: "DMRG_OK", -1: "DMRG_EINVAL", -2: "DMRG_ENOMEM", -3: "DMRG_EHIP",
          -4: "DMRG_ENONFINITE", -5: "DMRG_ESTATE", -6: "DMRG_EIO", 1: "DMRG_WNOTCONV"}
DMRG_WNOTCONV = 1
STATUS_CODE = {v: k for k, v in STATUS.items()}

# exported symbols (kept in sync with include/dmrgtst.h; checked by the CPU tests)
SYMBOLS = [
    "dmrg_create", "dmrg_destroy", "dmrg_psi_layout", "dmrg_flops", "dmrg_flops_executed",
    "dmrg_set_precision", "dmrg_set_check_finite", "dmrg_plan_stats",
    "dmrg_set_stream", "dmrg_matvec", "dmrg_matvec_noalloc", "dmrg_krylov_expm", "dmrg_tst_targets", "dmrg_set_graph",
    "dmrg_set_gemm", "dmrg_get_gemm", "dmrg_autotune", "dmrg_autotune_cached",
    "dmrg_batch_autotune_cached", "dmrg_tune_key", "dmrg_tune_cache_lookup",
    "dmrg_tune_cache_store",
    "dmrg_batch_create", "dmrg_batch_destroy", "dmrg_batch_set_graph", "dmrg_batch_tst_targets",
    "dmrg_batch_set_gemm", "dmrg_batch_autotune", "dmrg_profile_matvec",
    "dmrg_tst_chains", "dmrg_batch_tst_chains", "dmrg_ground_state", "dmrg_density_truncate",
    "dmrg_wft_create", "dmrg_wft_apply", "dmrg_wft_destroy", "dmrg_apply_local",
    "dmrg_expect_local",
    "dmrg_strerror", "dmrg_last_error",
]


class dmrg_op(C.Structure):
    _fields_ = [("dq", C.c_int32 * 2), ("blocks", C.POINTER(C.c_double))]


class dmrg_half(C.Structure):
    _fields_ = [("nsec", C.c_int32), ("qn", C.POINTER(C.c_int32)), ("dim", C.POINTER(C.c_int32)),
                ("H", C.POINTER(C.c_double)), ("nop", C.c_int32), ("ops", C.POINTER(dmrg_op))]


class dmrg_term(C.Structure):
    _fields_ = [("coef", C.c_double), ("opS", C.c_int32), ("transS", C.c_int32),
                ("opE", C.c_int32), ("transE", C.c_int32), ("fermionic", C.c_int32)]


class dmrg_bond(C.Structure):
    _fields_ = [("opS", C.c_int32 * 2), ("opE", C.c_int32 * 2), ("t", C.c_double)]


class dmrg_problem(C.Structure):
    _fields_ = [("S", dmrg_half), ("E", dmrg_half), ("target", C.c_int32 * 2),
                ("nbond", C.c_int32), ("bonds", C.POINTER(dmrg_bond)),
                ("nterm", C.c_int32), ("terms", C.POINTER(dmrg_term))]


class dmrg_wft_desc(C.Structure):
    _fields_ = [("n_esub", C.c_int32), ("esub", C.POINTER(C.c_int32)), ("nr", C.c_int32),
                ("r_dim", C.POINTER(C.c_int32)), ("r_to_enew", C.POINTER(C.c_int32)),
                ("kept", C.POINTER(C.c_int32)), ("n_ssub", C.c_int32),
                ("ssub", C.POINTER(C.c_int32)), ("ns_new", C.c_int32),
                ("s_new_qn", C.POINTER(C.c_int32)), ("s_new_dim", C.POINTER(C.c_int32)),
                ("ne_new", C.c_int32), ("e_new_qn", C.POINTER(C.c_int32)),
                ("e_new_dim", C.POINTER(C.c_int32))]


class dmrg_plan_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nblk", C.c_int32), ("flops", C.c_double),
                ("flops_executed", C.c_double), ("create_bytes", C.c_int64),
                ("krylov_bytes", C.c_int64)]


class dmrg_krylov_info(C.Structure):
    _fields_ = [("k_eff", C.c_int32), ("k_eff_min", C.c_int32), ("beta0", C.c_double),
                ("beta_last", C.c_double), ("err_est", C.c_double), ("breakdown", C.c_int32),
                ("converged", C.c_int32), ("k_eff_steps", C.POINTER(C.c_int32))]

    def as_dict(self, nsteps: int = 0):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "k_eff_steps"}
        if nsteps and self.k_eff_steps:
            d["k_eff_steps"] = [int(self.k_eff_steps[i]) for i in range(nsteps)]
        return d


def _info(nsteps: int = 0):
    """A zero-initialised info struct with a per-step array of nsteps entries (kept alive on
    the struct)."""
    inf = dmrg_krylov_info()
    if nsteps > 0:
        arr = (C.c_int32 * nsteps)()
        inf._steps = arr
        inf.k_eff_steps = C.cast(arr, C.POINTER(C.c_int32))
    return inf


_lib = None


def load(path: str = LIB_PATH):
    """Loads libdmrgtst.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_1103_5391_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    lib.dmrg_create.argtypes = [P(dmrg_problem), vp, P(vp)]
    lib.dmrg_destroy.argtypes = [vp]
    lib.dmrg_destroy.restype = None
    lib.dmrg_psi_layout.argtypes = [vp, P(i64), P(i32), P(i64), P(i32), P(i32), P(i32), P(i32)]
    lib.dmrg_flops.argtypes = [vp, P(dbl)]
    lib.dmrg_flops_executed.argtypes = [vp, P(dbl)]
    lib.dmrg_set_check_finite.argtypes = [vp, i32]
    lib.dmrg_plan_stats.argtypes = [P(dmrg_problem), i32, P(dmrg_plan_info)]
    lib.dmrg_set_precision.argtypes = [vp, i32]
    lib.dmrg_set_stream.argtypes = [vp, vp]
    lib.dmrg_matvec.argtypes = [vp, vp, vp, i32]
    lib.dmrg_matvec_noalloc.argtypes = [vp, vp, vp, i32]
    lib.dmrg_krylov_expm.argtypes = [vp, vp, vp, dbl, i32, i32, P(dmrg_krylov_info)]
    lib.dmrg_tst_targets.argtypes = [vp, vp, dbl, i32, vp, P(dbl), P(dmrg_krylov_info)]
    lib.dmrg_set_graph.argtypes = [vp, i32]
    lib.dmrg_set_gemm.argtypes = [vp, i32]
    lib.dmrg_get_gemm.argtypes = [vp, P(i32)]
    lib.dmrg_autotune.argtypes = [vp, i32, P(dbl)]
    lib.dmrg_batch_set_gemm.argtypes = [vp, i32]
    lib.dmrg_batch_autotune.argtypes = [vp, i32, P(dbl)]
    lib.dmrg_autotune_cached.argtypes = [vp, C.c_char_p, i32, P(dbl), P(i32)]
    lib.dmrg_batch_autotune_cached.argtypes = [vp, C.c_char_p, i32, P(dbl), P(i32)]
    lib.dmrg_tune_key.argtypes = [P(dmrg_problem), i32, C.c_char_p, C.c_char_p, i64, P(i64)]
    lib.dmrg_tune_cache_lookup.argtypes = [C.c_char_p, C.c_char_p, P(i32), P(dbl), P(i32)]
    lib.dmrg_tune_cache_store.argtypes = [C.c_char_p, C.c_char_p, i32, P(dbl)]
    lib.dmrg_batch_create.argtypes = [P(vp), i32, P(vp)]
    lib.dmrg_batch_set_graph.argtypes = [vp, i32]
    lib.dmrg_batch_destroy.argtypes = [vp]
    lib.dmrg_batch_destroy.restype = None
    lib.dmrg_batch_tst_targets.argtypes = [vp, P(vp), dbl, i32, P(vp), P(dbl),
                                           P(dmrg_krylov_info)]
    lib.dmrg_profile_matvec.argtypes = [vp, vp, vp, i32, P(dbl)]
    lib.dmrg_tst_chains.argtypes = [vp, P(vp), dbl, i32, P(vp), P(dbl), P(dmrg_krylov_info)]
    lib.dmrg_ground_state.argtypes = [vp, vp, vp, i32, i32, dbl, P(dbl), P(i32), P(dmrg_krylov_info)]
    lib.dmrg_density_truncate.argtypes = [vp, P(vp), P(dbl), i32, i32, vp, vp, P(i32), P(dbl)]
    lib.dmrg_batch_tst_chains.argtypes = [vp, P(vp), dbl, i32, P(vp), P(dbl),
                                          P(dmrg_krylov_info)]
    lib.dmrg_wft_create.argtypes = [vp, P(dmrg_wft_desc), P(vp), P(vp), P(i64)]
    lib.dmrg_wft_apply.argtypes = [vp, vp, i32, P(vp), P(vp), P(dbl)]
    lib.dmrg_wft_destroy.argtypes = [vp]
    lib.dmrg_apply_local.argtypes = [vp, vp, i32, P(dmrg_term), vp, vp]
    lib.dmrg_expect_local.argtypes = [vp, i32, P(dmrg_term), vp, P(dbl), P(dbl)]
    lib.dmrg_strerror.argtypes = [i32]
    lib.dmrg_strerror.restype = C.c_char_p
    lib.dmrg_last_error.argtypes = [vp]
    lib.dmrg_last_error.restype = C.c_char_p
    for s in SYMBOLS:
        if s not in ("dmrg_destroy", "dmrg_batch_destroy", "dmrg_strerror", "dmrg_last_error"):
            getattr(lib, s).restype = C.c_int
    _lib = lib
    return lib


class DmrgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(rc: int, handle=None):
    """Raises on an error status (negative); warnings (positive) are left to the caller."""
    if rc < 0:
        lib = load()
        msg = lib.dmrg_last_error(handle).decode()
        raise DmrgError(rc, msg or lib.dmrg_strerror(rc).decode())


def _dptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))


def _half_to_c(half, keep: list) -> dmrg_half:
    sp = half.space
    qn = np.ascontiguousarray(sp.qn, dtype=np.int32).reshape(-1)
    dim = np.ascontiguousarray(sp.dim, dtype=np.int32)
    H = np.concatenate([np.asarray(h, dtype=np.float64).reshape(-1, order="F") for h in half.H])
    ops = (dmrg_op * max(1, len(half.ops)))()
    for i, op in enumerate(half.ops):
        # the ABI wants one block for every source sector whose image exists (zeros if absent)
        parts = []
        for p in range(len(dim)):
            p2 = sp.shift(p, op.dq)
            if p2 is None:
                continue
            blk = op.blocks.get(p)
            if blk is None:
                blk = np.zeros((int(dim[p2]), int(dim[p])))
            parts.append(np.asarray(blk, dtype=np.float64).reshape(-1, order="F"))
        data = np.concatenate(parts) if parts else np.zeros(1)
        keep.append(data)
        ops[i].dq[0], ops[i].dq[1] = int(op.dq[0]), int(op.dq[1])
        ops[i].blocks = _dptr(data, C.c_double)
    keep.extend([qn, dim, H, ops])
    h = dmrg_half()
    h.nsec = len(dim)
    h.qn = _dptr(qn, C.c_int32)
    h.dim = _dptr(dim, C.c_int32)
    h.H = _dptr(H, C.c_double)
    h.nop = len(half.ops)
    h.ops = ops
    return h


def problem_to_c(pb, extra_terms=()):
    """C struct for an inputs.Problem (plus optional generic terms); returns (struct, keepalive)."""
    keep = []
    c = dmrg_problem()
    c.S = _half_to_c(pb.S, keep)
    c.E = _half_to_c(pb.E, keep)
    c.target[0], c.target[1] = int(pb.target[0]), int(pb.target[1])
    bonds = (dmrg_bond * max(1, len(pb.bonds)))()
    for i, b in enumerate(pb.bonds):
        bonds[i].opS[0], bonds[i].opS[1] = int(b.opS[0]), int(b.opS[1])
        bonds[i].opE[0], bonds[i].opE[1] = int(b.opE[0]), int(b.opE[1])
        bonds[i].t = float(b.t)
    c.nbond = len(pb.bonds)
    c.bonds = bonds
    terms = (dmrg_term * max(1, len(extra_terms)))()
    for i, t in enumerate(extra_terms):
        terms[i].coef, terms[i].opS, terms[i].transS = float(t[0]), int(t[1]), int(t[2])
        terms[i].opE, terms[i].transE, terms[i].fermionic = int(t[3]), int(t[4]), int(t[5])
    c.nterm = len(extra_terms)
    c.terms = terms
    keep.extend([bonds, terms])
    return c, keep


def _tensor_ptr(t, n2: int, count: int = 1):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous() and t.numel() >= n2 * count):
        raise ValueError("expected a contiguous float64 GPU tensor of at least "
                         f"{n2 * count} elements")
    return C.c_void_p(t.data_ptr())


def dmrg_create(pb, stream=None, extra_terms=()):
    """Creates a handle for an inputs.Problem; returns a Handle."""
    lib = load()
    cpb, keep = problem_to_c(pb, extra_terms)
    h = C.c_void_p()
    rc = lib.dmrg_create(C.byref(cpb), _stream_ptr(stream), C.byref(h))
    if rc != 0:
        raise DmrgError(rc, lib.dmrg_last_error(None).decode())
    return Handle(h)


def plan_stats(pb, kdim: int = 15, extra_terms=()) -> dict:
    """Host-only planning of a problem (no GPU needed): n, block count, algorithmic and executed
    flops, device bytes of dmrg_create and of a first Krylov call with kdim vectors."""
    lib = load()
    cpb, keep = problem_to_c(pb, extra_terms)
    st = dmrg_plan_info()
    rc = lib.dmrg_plan_stats(C.byref(cpb), int(kdim), C.byref(st))
    if rc != 0:
        raise DmrgError(rc, lib.dmrg_last_error(None).decode())
    return {f: getattr(st, f) for f, _ in st._fields_}


_TUNE_FIELDS = ("stage1_register", "stage1_lds", "stage2_register", "stage2_lds",
                "stage1_narrow", "stage2_narrow", "stage1_x", "stage2_x", "stage1_k", "stage2_k")


def _tune_dict(out, variant, hit=None):
    d = {f: float(v) for f, v in zip(_TUNE_FIELDS, out)}
    d["variant"] = int(variant)
    if hit is not None:
        d["cached"] = bool(hit)
    return d


def _path_bytes(path) -> bytes:
    return os.fsencode(os.fspath(path))


def tune_key(pb, precision: int = DMRG_FP64, arch: str = "gfx950", extra_terms=()) -> str:
    """Host-only key of a problem in the autotuner's cache (no GPU needed)."""
    lib = load()
    cpb, keep = problem_to_c(pb, extra_terms)
    n = C.c_int64()
    a = arch.encode()
    rc = lib.dmrg_tune_key(C.byref(cpb), int(precision), a, None, 0, C.byref(n))
    if rc != 0:
        raise DmrgError(rc, lib.dmrg_last_error(None).decode())
    buf = C.create_string_buffer(n.value + 1)
    rc = lib.dmrg_tune_key(C.byref(cpb), int(precision), a, buf, n.value + 1, C.byref(n))
    if rc != 0:
        raise DmrgError(rc, lib.dmrg_last_error(None).decode())
    return buf.value.decode()


def tune_cache_lookup(path, key: str):
    """Entry of key in the cache file at path as a dict (variant, timings), or None."""
    lib = load()
    v, found = C.c_int32(), C.c_int32()
    ms = np.zeros(10)
    rc = lib.dmrg_tune_cache_lookup(_path_bytes(path), key.encode(), C.byref(v),
                                    _dptr(ms, C.c_double), C.byref(found))
    if rc != 0:
        raise DmrgError(rc, lib.dmrg_last_error(None).decode())
    return _tune_dict(ms, v.value) if found.value else None


def tune_cache_store(path, key: str, variant: int, ms=None):
    """Adds or replaces the entry of key in the cache file at path."""
    lib = load()
    arr = None if ms is None else np.ascontiguousarray(ms, dtype=np.float64)
    if arr is not None and arr.size != 10:
        raise ValueError("ms must hold 10 timings")
    rc = lib.dmrg_tune_cache_store(_path_bytes(path), key.encode(), int(variant),
                                   None if arr is None else _dptr(arr, C.c_double))
    if rc != 0:
        raise DmrgError(rc, lib.dmrg_last_error(None).decode())


class Handle:
    def __init__(self, h: C.c_void_p):
        self.h = h
        self.lib = load()
        n, nb = C.c_int64(), C.c_int32()
        _check(self.lib.dmrg_psi_layout(h, C.byref(n), C.byref(nb), None, None, None, None, None), h)
        self.n, self.nblk = int(n.value), int(nb.value)

    def dmrg_destroy(self):
        if self.h:
            self.lib.dmrg_destroy(self.h)
            self.h = None

    destroy = dmrg_destroy

    def __del__(self):
        try:
            self.dmrg_destroy()
        except Exception:
            pass

    def dmrg_psi_layout(self):
        nb = self.nblk
        off = np.zeros(nb, np.int64)
        arr = [np.zeros(nb, np.int32) for _ in range(4)]
        _check(self.lib.dmrg_psi_layout(self.h, None, None, _dptr(off, C.c_int64),
                                        *[_dptr(a, C.c_int32) for a in arr]), self.h)
        return dict(n=self.n, off=off, rows=arr[0], cols=arr[1], secS=arr[2], secE=arr[3])

    psi_layout = dmrg_psi_layout

    def dmrg_flops(self) -> float:
        f = C.c_double()
        _check(self.lib.dmrg_flops(self.h, C.byref(f)), self.h)
        return f.value

    flops = dmrg_flops

    def dmrg_flops_executed(self) -> float:
        f = C.c_double()
        _check(self.lib.dmrg_flops_executed(self.h, C.byref(f)), self.h)
        return f.value

    flops_executed = dmrg_flops_executed

    def dmrg_set_check_finite(self, enable: bool):
        _check(self.lib.dmrg_set_check_finite(self.h, int(bool(enable))), self.h)

    set_check_finite = dmrg_set_check_finite

    def dmrg_set_precision(self, prec: int):
        _check(self.lib.dmrg_set_precision(self.h, int(prec)), self.h)

    set_precision = dmrg_set_precision

    def dmrg_set_stream(self, stream):
        _check(self.lib.dmrg_set_stream(self.h, _stream_ptr(stream)), self.h)

    set_stream = dmrg_set_stream

    def dmrg_matvec(self, x, y, nvec: int = 1):
        n2 = 2 * self.n
        _check(self.lib.dmrg_matvec(self.h, _tensor_ptr(x, n2, nvec), _tensor_ptr(y, n2, nvec),
                                    int(nvec)), self.h)

    matvec = dmrg_matvec

    def dmrg_matvec_noalloc(self, x, y, nvec: int = 1):
        """As dmrg_matvec, with the intermediate in the library's per-GPU scratch (no device
        allocation in the call; the problem's intermediate must fit the scratch)."""
        n2 = 2 * self.n
        _check(self.lib.dmrg_matvec_noalloc(self.h, _tensor_ptr(x, n2, nvec),
                                            _tensor_ptr(y, n2, nvec), int(nvec)), self.h)

    matvec_noalloc = dmrg_matvec_noalloc

    def dmrg_krylov_expm(self, x, y, tau: float, kdim: int, nsteps: int = 1, info: bool = True):
        """y = exp(-i tau H)^nsteps x; returns the info dict (with k_eff_steps per step)."""
        n2 = 2 * self.n
        inf = _info(nsteps)
        _check(self.lib.dmrg_krylov_expm(self.h, _tensor_ptr(x, n2), _tensor_ptr(y, n2),
                                         float(tau), int(kdim), int(nsteps),
                                         C.byref(inf) if info else None), self.h)
        return inf.as_dict(nsteps) if info else None

    krylov_expm = dmrg_krylov_expm

    def dmrg_tst_targets(self, phi, tau: float, kdim: int, targets, info: bool = True):
        n2 = 2 * self.n
        w = np.zeros(5)
        inf = dmrg_krylov_info()
        _check(self.lib.dmrg_tst_targets(self.h, _tensor_ptr(phi, n2), float(tau), int(kdim),
                                         _tensor_ptr(targets, n2, 4), _dptr(w, C.c_double),
                                         C.byref(inf) if info else None), self.h)
        return w, (inf.as_dict() if info else None)

    tst_targets = dmrg_tst_targets

    def dmrg_tst_chains(self, phis, tau: float, kdim: int, targets, info: bool = True):
        """4-RHS mode: targets[k] = exp(-i tau H) phis[k] for four device vectors, in common
        launches."""
        n2 = 2 * self.n
        ph = (C.c_void_p * 4)(*[_tensor_ptr(p, n2).value for p in phis])
        tg = (C.c_void_p * 4)(*[_tensor_ptr(t, n2).value for t in targets])
        w = np.zeros(5)
        infos = (dmrg_krylov_info * 4)()
        _check(self.lib.dmrg_tst_chains(self.h, ph, float(tau), int(kdim), tg, _dptr(w, C.c_double),
                                        infos if info else None), self.h)
        return w, ([i.as_dict() for i in infos] if info else None)

    tst_chains = dmrg_tst_chains

    def dmrg_ground_state(self, x0, y, kdim: int, max_restarts: int = 20, tol: float = 1e-10,
                          info: bool = True):
        """Restarted Lanczos ground state: y = unit Ritz vector; returns (energy, bases used,
        info)."""
        n2 = 2 * self.n
        e = C.c_double()
        used = C.c_int32()
        inf = _info(max_restarts)
        rc = self.lib.dmrg_ground_state(self.h, _tensor_ptr(x0, n2), _tensor_ptr(y, n2), int(kdim),
                                        int(max_restarts), float(tol), C.byref(e), C.byref(used),
                                        C.byref(inf) if info else None)
        _check(rc, self.h)      # DMRG_WNOTCONV: returned, info["converged"] = 0
        return e.value, used.value, (inf.as_dict(used.value) if info else None)

    ground_state = dmrg_ground_state

    def dmrg_density_truncate(self, vecs, weights, keep: int, evals, evecs):
        """Density matrix of the targets and its truncation to `keep` states: fills the device
        buffers evals (sum d) and evecs (sum 2 d^2); returns (kept per sector, truncation error)."""
        n2 = 2 * self.n
        lay = self.psi_layout()
        rows = [int(r) for r in lay["rows"]]
        ne, nv2 = sum(rows), sum(2 * r * r for r in rows)
        ph = (C.c_void_p * len(vecs))(*[_tensor_ptr(v, n2).value for v in vecs])
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
        kept = np.zeros(len(rows), dtype=np.int32)
        err = C.c_double()
        _check(self.lib.dmrg_density_truncate(self.h, ph, _dptr(w, C.c_double), len(vecs), int(keep),
                                              _tensor_ptr(evals, ne), _tensor_ptr(evecs, nv2),
                                              _dptr(kept, C.c_int32), C.byref(err)), self.h)
        return kept, err.value

    density_truncate = dmrg_density_truncate

    def dmrg_apply_local(self, dst: "Handle", terms, x, y):
        """y (dst's layout) = sum of terms applied to x; a term is (coef, opS, transS, opE,
        transE, fermionic) with op indices into this handle's half operators (-1: identity)."""
        ct = _terms_to_c(terms)
        _check(self.lib.dmrg_apply_local(self.h, dst.h, len(terms), ct, _tensor_ptr(x, 2 * self.n),
                                         _tensor_ptr(y, 2 * dst.n)), self.h)

    apply_local = dmrg_apply_local

    def dmrg_expect_local(self, terms, x) -> complex:
        """<x| sum of terms |x> (terms that keep the sector)."""
        ct = _terms_to_c(terms)
        re, im = C.c_double(), C.c_double()
        _check(self.lib.dmrg_expect_local(self.h, len(terms), ct, _tensor_ptr(x, 2 * self.n),
                                          C.byref(re), C.byref(im)), self.h)
        return complex(re.value, im.value)

    expect_local = dmrg_expect_local

    def dmrg_wft_create(self, mv, W):
        """Plans a move of the centre (wave-function transformation) described by mv (an
        inputs.WftMove: sector tables of the move); W: per R sector a device tensor of
        2 d_E' d_R doubles (W_r column-major, real then imaginary parts)."""
        return Wft(self, mv, W)

    wft_create = dmrg_wft_create

    def dmrg_set_graph(self, enable: bool):
        _check(self.lib.dmrg_set_graph(self.h, int(bool(enable))), self.h)

    set_graph = dmrg_set_graph

    def dmrg_set_gemm(self, variant: int):
        _check(self.lib.dmrg_set_gemm(self.h, int(variant)), self.h)

    set_gemm = dmrg_set_gemm

    def dmrg_get_gemm(self) -> int:
        v = C.c_int32()
        _check(self.lib.dmrg_get_gemm(self.h, C.byref(v)), self.h)
        return v.value

    get_gemm = dmrg_get_gemm

    def dmrg_autotune(self, reps: int = 10, cache=None):
        """Times the kernel families of each stage, keeps the fastest; returns the timings (ms)
        and the chosen variant bits.  cache: None, or the path of a JSON tuning cache that is
        consulted first (a hit applies the stored choice without timing; "cached" in the result
        tells which) and updated after a miss."""
        out = np.zeros(10)
        if cache is None:
            _check(self.lib.dmrg_autotune(self.h, int(reps), _dptr(out, C.c_double)), self.h)
            return _tune_dict(out, self.get_gemm())
        hit = C.c_int32()
        _check(self.lib.dmrg_autotune_cached(self.h, _path_bytes(cache), int(reps),
                                             _dptr(out, C.c_double), C.byref(hit)), self.h)
        return _tune_dict(out, self.get_gemm(), hit.value)

    autotune = dmrg_autotune

    def dmrg_profile_matvec(self, x, y, reps: int = 10):
        """Average ms of the two block-product launches and their algorithmic flops."""
        n2 = 2 * self.n
        out = np.zeros(4)
        _check(self.lib.dmrg_profile_matvec(self.h, _tensor_ptr(x, n2), _tensor_ptr(y, n2),
                                            int(reps), _dptr(out, C.c_double)), self.h)
        return dict(ms_stage1=out[0], ms_stage2=out[1], flops_stage1=out[2], flops_stage2=out[3])

    profile_matvec = dmrg_profile_matvec


class Batch:
    """Batched time-step targeting over independent handles."""

    def __init__(self, handles):
        self.lib = load()
        self.handles = list(handles)
        arr = (C.c_void_p * len(self.handles))(*[h.h for h in self.handles])
        b = C.c_void_p()
        rc = self.lib.dmrg_batch_create(arr, len(self.handles), C.byref(b))
        if rc != 0:
            _check(rc, self.handles[0].h)
        self.b = b

    def dmrg_batch_set_graph(self, enable: bool):
        _check(self.lib.dmrg_batch_set_graph(self.b, int(bool(enable))), self.handles[0].h)

    set_graph = dmrg_batch_set_graph

    def dmrg_batch_set_gemm(self, variant: int):
        _check(self.lib.dmrg_batch_set_gemm(self.b, int(variant)), self.handles[0].h)

    set_gemm = dmrg_batch_set_gemm

    def dmrg_batch_autotune(self, reps: int = 5, cache=None):
        """As Handle.autotune, for the merged launches of the batch."""
        out = np.zeros(10)
        if cache is None:
            _check(self.lib.dmrg_batch_autotune(self.b, int(reps), _dptr(out, C.c_double)),
                   self.handles[0].h)
            return {f: float(v) for f, v in zip(_TUNE_FIELDS, out)}
        hit = C.c_int32()
        _check(self.lib.dmrg_batch_autotune_cached(self.b, _path_bytes(cache), int(reps),
                                                   _dptr(out, C.c_double), C.byref(hit)),
               self.handles[0].h)
        d = {f: float(v) for f, v in zip(_TUNE_FIELDS, out)}
        d["cached"] = bool(hit.value)
        return d

    autotune = dmrg_batch_autotune

    def dmrg_batch_tst_targets(self, phis, tau: float, kdim: int, targets, info: bool = True):
        cnt = len(self.handles)
        ph = (C.c_void_p * cnt)(*[_tensor_ptr(p, 2 * h.n).value for p, h in zip(phis, self.handles)])
        tg = (C.c_void_p * cnt)(*[_tensor_ptr(t, 2 * h.n, 4).value for t, h in zip(targets, self.handles)])
        w = np.zeros(5)
        infos = (dmrg_krylov_info * cnt)()
        rc = self.lib.dmrg_batch_tst_targets(self.b, ph, float(tau), int(kdim), tg,
                                             _dptr(w, C.c_double), infos if info else None)
        if rc != 0:
            _check(rc, self.handles[0].h)
        return w, ([i.as_dict() for i in infos] if info else None)

    batch_tst_targets = dmrg_batch_tst_targets

    def dmrg_batch_tst_chains(self, phis, tau: float, kdim: int, targets, info: bool = True):
        """4-RHS mode of every superblock: phis, targets: 4 x count device vectors, chain k of
        superblock i at [4 i + k]."""
        cnt = 4 * len(self.handles)
        hs = [h for h in self.handles for _ in range(4)]
        ph = (C.c_void_p * cnt)(*[_tensor_ptr(p, 2 * h.n).value for p, h in zip(phis, hs)])
        tg = (C.c_void_p * cnt)(*[_tensor_ptr(t, 2 * h.n).value for t, h in zip(targets, hs)])
        w = np.zeros(5)
        infos = (dmrg_krylov_info * cnt)()
        rc = self.lib.dmrg_batch_tst_chains(self.b, ph, float(tau), int(kdim), tg,
                                            _dptr(w, C.c_double), infos if info else None)
        if rc != 0:
            _check(rc, self.handles[0].h)
        return w, ([i.as_dict() for i in infos] if info else None)

    batch_tst_chains = dmrg_batch_tst_chains

    def dmrg_batch_destroy(self):
        if self.b:
            self.lib.dmrg_batch_destroy(self.b)
            self.b = None

    destroy = dmrg_batch_destroy

    def __del__(self):
        try:
            self.dmrg_batch_destroy()
        except Exception:
            pass


def _terms_to_c(terms):
    ct = (dmrg_term * max(1, len(terms)))()
    for i, t in enumerate(terms):
        ct[i].coef, ct[i].opS, ct[i].transS = float(t[0]), int(t[1]), int(t[2])
        ct[i].opE, ct[i].transE, ct[i].fermionic = int(t[3]), int(t[4]), int(t[5])
    return ct


def _i32(rows) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1))


class Wft:
    """A planned move of the centre (dmrg_wft_create / dmrg_wft_apply / dmrg_wft_destroy)."""

    def __init__(self, handle: "Handle", mv, W):
        self.handle, self.lib, self.w = handle, handle.lib, C.c_void_p()
        S, E = mv.layout.S.space, mv.layout.E.space
        ssub = [(b, a, pp, off) for (b, a), (pp, off) in sorted(mv.ssub.items())]
        self._keep = t = {
            "esub": _i32(mv.esub), "r_dim": _i32(mv.r_dim), "r_to_enew": _i32(mv.r_to_enew),
            "kept": _i32(mv.kept), "ssub": _i32(ssub), "s_qn": _i32(S.qn), "s_dim": _i32(S.dim),
            "e_qn": _i32(E.qn), "e_dim": _i32(E.dim)}
        d = dmrg_wft_desc(len(mv.esub), _dptr(t["esub"], C.c_int32), len(mv.r_dim),
                          _dptr(t["r_dim"], C.c_int32), _dptr(t["r_to_enew"], C.c_int32),
                          _dptr(t["kept"], C.c_int32), len(ssub), _dptr(t["ssub"], C.c_int32),
                          len(S.dim), _dptr(t["s_qn"], C.c_int32), _dptr(t["s_dim"], C.c_int32),
                          len(E.dim), _dptr(t["e_qn"], C.c_int32), _dptr(t["e_dim"], C.c_int32))
        wp = (C.c_void_p * max(1, len(W)))(*[_tensor_ptr(x, x.numel()).value for x in W])
        n_new = C.c_int64()
        _check(self.lib.dmrg_wft_create(handle.h, C.byref(d), wp, C.byref(self.w), C.byref(n_new)),
               handle.h)
        self.n_new = n_new.value

    def apply(self, U, xs, ys) -> float:
        """y[v] = transformation of x[v] (device tensors of 2n and 2 n_new doubles), with U the
        eigenvector buffer of density_truncate; returns the algorithmic flops."""
        n2, m2 = 2 * self.handle.n, 2 * self.n_new
        px = (C.c_void_p * len(xs))(*[_tensor_ptr(x, n2).value for x in xs])
        py = (C.c_void_p * len(ys))(*[_tensor_ptr(y, m2).value for y in ys])
        fl = C.c_double()
        nu = sum(2 * int(r) * int(r) for r in self.handle.psi_layout()["rows"])
        _check(self.lib.dmrg_wft_apply(self.w, _tensor_ptr(U, nu), len(xs), px, py, C.byref(fl)),
               self.handle.h)
        return fl.value

    def destroy(self):
        if self.w:
            self.lib.dmrg_wft_destroy(self.w)
            self.w = C.c_void_p()
