"""ctypes binding of libthc.so (C ABI in include/thc.h).

Argument marshalling only: tensors are passed as device pointers, the stream is torch's
current HIP stream, and every computation runs in the library's kernels.  There is no CPU
fallback: if the library is missing or the tensors are not on the GPU, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libthc.so")

THC_OK, THC_EINVAL, THC_ENOMEM, THC_EDEVICE, THC_ESINGULAR, THC_ENUMERIC, THC_ENOTCONV, THC_ESTATE, THC_EDIVERGED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
ERRNAMES = {0: "THC_OK", -1: "THC_EINVAL", -2: "THC_ENOMEM", -3: "THC_EDEVICE", -4: "THC_ESINGULAR",
            -5: "THC_ENUMERIC", -6: "THC_ENOTCONV", -7: "THC_ESTATE", -8: "THC_EDIVERGED"}
ITER_MIXED, ITER_RESTARTED, ITER_DIIS_DROPPED, ITER_LEARNED = 1, 2, 4, 8
# contraction chains (bits of Options.split_mask)
CHAIN_FUSED, CHAIN_ASSEMBLY, CHAIN_ALG45, CHAIN_ALG6, CHAIN_ALG7, CHAIN_SINGLES = (1 << k for k in range(6))
CHAIN_ALL = 0x3F

TERM_EQ28, TERM_EQ29, TERM_EQ31, TERM_EQ32, TERM_EQ35, TERM_EQ41, TERM_EQ38, TERM_EQ42 = (1 << k for k in range(8))
TERM_ALL = 0xFF
FLAG_UNFUSED_EXCHANGE = 1 << 0
TERMS = {"eq28": TERM_EQ28, "eq29": TERM_EQ29, "eq31": TERM_EQ31, "eq32+33": TERM_EQ32, "eq35": TERM_EQ35,
         "eq41": TERM_EQ41, "eq38": TERM_EQ38, "eq42": TERM_EQ42}

# exported symbols (kept in sync with include/thc.h; checked by the tests)
SYMBOLS = ["thc_create", "thc_build_factors", "thc_residual", "thc_residual_terms", "thc_iterate", "thc_history",
           "thc_history_precision", "thc_history_flags", "thc_checkpoint_bytes", "thc_save_checkpoint",
           "thc_load_checkpoint",
           "thc_energy",
           "thc_get_state", "thc_set_state", "thc_memory_bytes", "thc_plan",
           "thc_set_synthetic", "thc_synth_gamma", "thc_mp2_density", "thc_create_with_workspace", "thc_plan_query", "thc_synth_normals", "thc_synth_cholesky", "thc_synth_energies", "thc_cp_als", "thc_profile", "thc_profile_get", "thc_profile_flops", "thc_dgemm",
           "thc_last_error", "thc_destroy",
           "thc_guess_features", "thc_guess_apply", "thc_set_guess_network", "thc_set_shift", "thc_working", "thc_guess_targets",
           "thc_mlp_create", "thc_mlp_set_norm", "thc_mlp_fit_norm", "thc_mlp_get_norm", "thc_mlp_num_params", "thc_mlp_get_params", "thc_mlp_set_params",
           "thc_mlp_forward", "thc_mlp_forward_noalloc", "thc_mlp_loss_grad", "thc_mlp_train_step", "thc_mlp_infer", "thc_mlp_last_error",
           "thc_mlp_destroy"]
GUESS_FEATURES = 10
MLP_SCRATCH_BYTES = 32 << 20  # the allocation-free forward pass's fixed device array per GPU


class Options(C.Structure):
    _fields_ = [("o", C.c_int64), ("v", C.c_int64), ("nL", C.c_int64), ("nP", C.c_int64), ("nQ", C.c_int64),
                ("singles", C.c_int32), ("diis_max", C.c_int32), ("tol_energy", C.c_double),
                ("a_block", C.c_int64), ("i_chunk", C.c_int64), ("x_block", C.c_int64), ("x_chunk", C.c_int64),
                ("precision", C.c_int32), ("flags", C.c_int32), ("x7_chunk", C.c_int64), ("q_pairs", C.c_int64),
                ("q_jchunk", C.c_int64), ("split_mask", C.c_uint64), ("guess", C.c_int32), ("reserved", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("a_block", C.c_int64), ("alg1_splits", C.c_int64), ("alg1_tile", C.c_int64),
                ("x_block", C.c_int64), ("x_blocks", C.c_int64), ("i_chunk", C.c_int64), ("i_chunks", C.c_int64),
                ("h_generations", C.c_int64), ("h_tiles", C.c_int64), ("x_chunk", C.c_int64),
                ("x7_chunk", C.c_int64), ("x7_chunks", C.c_int64),
                ("exchange_fused", C.c_int32), ("lvv_resident", C.c_int32), ("quintic", C.c_int32),
                ("reserved", C.c_int32), ("q_pairs", C.c_int64), ("q_jchunk", C.c_int64), ("device_bytes", C.c_uint64)]


class SynthSpec(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("decay", C.c_double), ("coupling", C.c_double), ("gamma", C.c_double)]


FLAG_STREAM_LVV = 1 << 1
FLAG_PROGRESS = 1 << 2
FLAG_QUINTIC = 1 << 3
FLAG_QUARTIC = 1 << 4
FLAG_CHECK = 1 << 5


class ThcError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__(f"{ERRNAMES.get(rc, rc)}: {msg}")
        self.rc = rc


_lib = None


def load(path: str = LIB_PATH):
    """Loads libthc.so and declares the prototypes; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2111_11473_amd.build`")
    lib = C.CDLL(path)
    P, I64, D, VP = C.c_void_p, C.c_int64, C.c_double, C.c_void_p
    lib.thc_create.argtypes = [C.POINTER(Options), VP, C.POINTER(VP)]
    lib.thc_build_factors.argtypes = [VP, P, P, P, P]
    lib.thc_residual.argtypes = [VP, P, P, P, P, C.POINTER(D)]
    lib.thc_residual_terms.argtypes = [VP, P, P, C.c_uint32, P, P]
    lib.thc_iterate.argtypes = [VP, D, C.c_int, C.POINTER(C.c_int), C.POINTER(D)]
    lib.thc_history.argtypes = [VP, C.c_int, C.POINTER(D), C.POINTER(D), C.POINTER(D), C.POINTER(C.c_int)]
    lib.thc_energy.argtypes = [VP, C.POINTER(D)]
    lib.thc_history_precision.argtypes = [VP, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.thc_history_flags.argtypes = [VP, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.thc_checkpoint_bytes.argtypes = [VP, C.POINTER(C.c_size_t)]
    lib.thc_save_checkpoint.argtypes = [VP, VP, C.c_size_t]
    lib.thc_load_checkpoint.argtypes = [VP, VP, C.c_size_t]
    lib.thc_get_state.argtypes = [VP, P, P]
    lib.thc_set_state.argtypes = [VP, P, P]
    lib.thc_memory_bytes.argtypes = [VP, C.POINTER(C.c_size_t)]
    lib.thc_plan.argtypes = [VP, C.POINTER(PlanInfo)]
    lib.thc_set_synthetic.argtypes = [VP, C.POINTER(SynthSpec)]
    lib.thc_mp2_density.argtypes = [VP, P, P, P]
    lib.thc_create_with_workspace.argtypes = [C.POINTER(Options), VP, C.c_size_t, VP, C.POINTER(VP)]
    lib.thc_plan_query.argtypes = [C.POINTER(Options), C.c_int, C.c_uint64, C.POINTER(PlanInfo)]
    lib.thc_synth_gamma.argtypes = [VP, C.POINTER(D)]
    lib.thc_synth_normals.argtypes = [C.c_uint64, C.c_int32, C.c_uint64, I64, D, P, VP]
    lib.thc_synth_cholesky.argtypes = [C.c_uint64, I64, I64, I64, D, D, P, VP]
    lib.thc_synth_energies.argtypes = [C.c_uint64, I64, I64, C.POINTER(D)]
    lib.thc_cp_als.argtypes = [P, I64, I64, I64, I64, P, P, P, P, P, P, C.c_int, D, C.c_int, C.POINTER(D),
                               C.POINTER(C.c_int), VP]
    lib.thc_profile.argtypes = [VP, C.c_int]
    lib.thc_profile_get.argtypes = [VP, C.c_char_p, C.POINTER(D), C.POINTER(I64)]
    lib.thc_profile_flops.argtypes = [VP, C.POINTER(D), C.POINTER(D), C.POINTER(D)]
    lib.thc_dgemm.argtypes = [C.c_int, C.c_int, I64, I64, I64, D, P, I64, I64, P, I64, I64, D, P, I64, I64, I64, VP]
    lib.thc_last_error.argtypes = [VP]
    lib.thc_last_error.restype = C.c_char_p
    lib.thc_destroy.argtypes = [VP]
    lib.thc_destroy.restype = None
    lib.thc_guess_features.argtypes = [VP, P]
    lib.thc_guess_apply.argtypes = [VP, P, I64]
    lib.thc_set_guess_network.argtypes = [VP, VP]
    lib.thc_set_shift.argtypes = [VP, P]
    lib.thc_working.argtypes = [VP, P, P]
    lib.thc_guess_targets.argtypes = [VP, P, P, P, P, P]
    FP = C.POINTER(C.c_float)
    lib.thc_mlp_create.argtypes = [I64, I64, I64, C.c_uint64, VP, C.POINTER(VP)]
    lib.thc_mlp_set_norm.argtypes = [VP, FP, FP, FP, FP]
    lib.thc_mlp_fit_norm.argtypes = [VP, P, P, I64]
    lib.thc_mlp_get_norm.argtypes = [VP, FP, FP, FP, FP]
    lib.thc_mlp_num_params.argtypes = [VP, C.POINTER(I64)]
    lib.thc_mlp_get_params.argtypes = [VP, P]
    lib.thc_mlp_set_params.argtypes = [VP, P]
    lib.thc_mlp_forward.argtypes = [VP, P, I64, P]
    lib.thc_mlp_forward_noalloc.argtypes = [VP, P, I64, P]
    lib.thc_mlp_loss_grad.argtypes = [VP, P, P, I64, FP, P]
    lib.thc_mlp_train_step.argtypes = [VP, P, P, I64, C.c_float, FP]
    lib.thc_mlp_infer.argtypes = [VP, P, I64, P]
    lib.thc_mlp_last_error.argtypes = [VP]
    lib.thc_mlp_last_error.restype = C.c_char_p
    lib.thc_mlp_destroy.argtypes = [VP]
    lib.thc_mlp_destroy.restype = None
    for name in SYMBOLS:
        if name not in ("thc_last_error", "thc_destroy", "thc_mlp_last_error", "thc_mlp_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _ptr(t, n=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return C.c_void_p(t.data_ptr())


def _fptr(t, n=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def dgemm(A, B, C_out, transA=False, transB=False, alpha=1.0, beta=0.0):
    """C = alpha op(A) op(B) + beta C on the library's MFMA kernel (2-D or batched 3-D tensors)."""
    lib = load()
    if not (A.dim() == B.dim() == C_out.dim()) or A.dim() not in (2, 3):
        raise ValueError("A, B and C must all be 2-D, or all 3-D (a batch)")
    batched = A.dim() == 3
    Am, Bm, Cm = (A, B, C_out) if batched else (A[None], B[None], C_out[None])
    nb = Cm.shape[0]
    M, N = Cm.shape[1], Cm.shape[2]
    K = Am.shape[1] if transA else Am.shape[2]
    rows_a = Am.shape[2] if transA else Am.shape[1]
    k_b, cols_b = (Bm.shape[2], Bm.shape[1]) if transB else (Bm.shape[1], Bm.shape[2])
    if rows_a != M or cols_b != N or k_b != K:
        raise ValueError(f"op(A) is {rows_a} x {K} and op(B) {k_b} x {cols_b}, C is {M} x {N}")
    if Am.shape[0] not in (1, nb) or Bm.shape[0] not in (1, nb):
        raise ValueError("A and B must hold one matrix or as many as C")
    sA = Am.stride(0) if Am.shape[0] > 1 else 0
    sB = Bm.stride(0) if Bm.shape[0] > 1 else 0
    rc = lib.thc_dgemm(int(transA), int(transB), M, N, K, alpha, _ptr(A, name="A"), Am.shape[2], sA, _ptr(B, name="B"),
                       Bm.shape[2], sB, beta, _ptr(C_out, name="C"), N, Cm.stride(0), nb, _stream())
    if rc != 0:
        raise ThcError(rc, "thc_dgemm failed")
    return C_out


def make_options(o, v, nL, nP, nQ, singles=True, diis_max=8, tol_energy=1e-8, a_block=0, i_chunk=0, x_block=0,
                 x_chunk=0, flags=0, precision=0, x7_chunk=0, q_pairs=0, q_jchunk=0, split_mask=0, guess=0):
    return Options(o, v, nL, nP, nQ, int(singles), diis_max, tol_energy, a_block, i_chunk, x_block, x_chunk,
                   precision, flags, x7_chunk, q_pairs, q_jchunk, split_mask, guess, 0)


def plan_query(o, v, nL, nP, nQ, budget_bytes, synthetic=False, **kw):
    """The blocking and working memory the library would plan within budget_bytes (a dict of
    PlanInfo's fields); needs no GPU."""
    lib = load()
    opt = make_options(o, v, nL, nP, nQ, **kw)
    p = PlanInfo()
    rc = lib.thc_plan_query(C.byref(opt), int(bool(synthetic)), C.c_uint64(int(budget_bytes)), C.byref(p))
    if rc != 0:
        raise ThcError(rc, "thc_plan_query: no plan fits")
    return {name: getattr(p, name) for name, _ in PlanInfo._fields_}


def synth_normals(seed, stream_id, first, count, divisor=1.0):
    """Normals first .. first + count - 1 of generator stream stream_id, divided by divisor, made
    on the GPU (the same values as synth.normal)."""
    lib = load()
    out = torch.empty(count, dtype=torch.float64, device="cuda")
    rc = lib.thc_synth_normals(C.c_uint64(seed), stream_id, C.c_uint64(first), count, divisor, _ptr(out), _stream())
    if rc != 0:
        raise ThcError(rc, "thc_synth_normals failed")
    return out


def synth_cholesky(seed, n, K0, nK, decay, gamma):
    """Cholesky vectors K0 .. K0 + nK - 1 (nK x n x n, times gamma) made on the GPU."""
    lib = load()
    out = torch.empty((nK, n, n), dtype=torch.float64, device="cuda")
    rc = lib.thc_synth_cholesky(C.c_uint64(seed), n, K0, nK, decay, gamma, _ptr(out), _stream())
    if rc != 0:
        raise ThcError(rc, "thc_synth_cholesky failed")
    return out


def synth_energies(seed, o, v):
    """Orbital energies (o occupied, v virtual, each sorted) from the library's generator (host)."""
    lib = load()
    e = (C.c_double * (o + v))()
    rc = lib.thc_synth_energies(C.c_uint64(seed), o, v, e)
    if rc != 0:
        raise ThcError(rc, "thc_synth_energies failed")
    return list(e)


def cp_als(A, X, Y, Z, sweeps, w1=None, w2=None, w3=None, cg_tol=1e-12, cg_maxit=500, objective=True):
    """Weighted CP-ALS on the GPU: `sweeps` sweeps (X, Y, Z in turn) updating the float64 CUDA
    tensors X [I, n], Y [J, n], Z [K, n] in place for the array A [I, J, K] and optional weights.
    Returns (objective list of sweeps + 1 values or None, most CG iterations of one solve)."""
    lib = load()
    I, J, K = A.shape
    n = X.shape[1]
    if X.shape != (I, n) or Y.shape != (J, n) or Z.shape != (K, n):
        raise ValueError("factor shapes do not match A")
    obj = (C.c_double * (sweeps + 1))() if objective else None
    its = C.c_int(0)
    rc = lib.thc_cp_als(_ptr(A, name="A"), I, J, K, n, _ptr(w1, I, "w1"), _ptr(w2, J, "w2"), _ptr(w3, K, "w3"),
                        _ptr(X, name="X"), _ptr(Y, name="Y"), _ptr(Z, name="Z"), int(sweeps), float(cg_tol),
                        int(cg_maxit), obj, C.byref(its), _stream())
    if rc != 0:
        raise ThcError(rc, "thc_cp_als failed")
    return (list(obj) if objective else None), its.value


class THC:
    """One THC-CCSD problem on the current GPU (all tensors float64, CUDA, contiguous)."""

    def __init__(self, o, v, nL, nP, nQ, singles=True, diis_max=8, tol_energy=1e-8, a_block=0, i_chunk=0,
                 x_block=0, x_chunk=0, flags=0, precision=0, x7_chunk=0, q_pairs=0, q_jchunk=0, split_mask=0,
                 guess=0, workspace=None):
        """workspace: None (the library allocates its working memory), or a CUDA tensor whose
        memory the library uses instead (thc_create_with_workspace; kept referenced here)."""
        self.lib = load()
        self.o, self.v, self.nL, self.nP, self.nQ = o, v, nL, nP, nQ
        self.singles = bool(singles)
        opt = make_options(o, v, nL, nP, nQ, singles, diis_max, tol_energy, a_block, i_chunk, x_block, x_chunk,
                           flags, precision, x7_chunk, q_pairs, q_jchunk, split_mask, guess)
        h = C.c_void_p()
        self.workspace = workspace
        if workspace is None:
            rc = self.lib.thc_create(C.byref(opt), _stream(), C.byref(h))
        else:
            if not isinstance(workspace, torch.Tensor) or workspace.device.type != "cuda" or not workspace.is_contiguous():
                raise TypeError("workspace must be a contiguous CUDA tensor")
            rc = self.lib.thc_create_with_workspace(C.byref(opt), C.c_void_p(workspace.data_ptr()),
                                                    workspace.numel() * workspace.element_size(), _stream(), C.byref(h))
        if rc != 0:
            raise ThcError(rc, "thc_create failed")
        self.ctx = h

    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.thc_last_error(self.ctx)
            raise ThcError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.thc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up -------------------------------------------------------------------------
    def build_factors(self, L, eps, Xo, Xv, xo, xv):
        """Uploads nothing itself: L, eps and the factors must already be GPU tensors.
        Returns the MP2-guess core Z0 (nP x nP)."""
        o, v, n = self.o, self.v, self.o + self.v
        X = torch.cat([Xo.reshape(-1), Xv.reshape(-1), xo.reshape(-1), xv.reshape(-1)]).contiguous()
        Z = torch.empty((self.nP, self.nP), dtype=torch.float64, device=L.device)
        rc = self.lib.thc_build_factors(self.ctx, _ptr(L, self.nL * n * n, "L"), _ptr(eps, n, "eps"),
                                        _ptr(X, o * self.nP + v * self.nP + (o + v) * self.nQ, "X"), _ptr(Z))
        self._check(rc, "thc_build_factors")
        return Z

    def set_synthetic(self, seed, decay, coupling=0.2, gamma=0.0):
        """Inputs generated on the GPU by the library (thc_set_synthetic); then build_synthetic()."""
        spec = SynthSpec(seed, decay, coupling, gamma)
        self._check(self.lib.thc_set_synthetic(self.ctx, C.byref(spec)), "thc_set_synthetic")

    def build_synthetic(self):
        """thc_build_factors on the generated inputs; returns the MP2-guess core Z0."""
        Z = torch.empty((self.nP, self.nP), dtype=torch.float64, device="cuda")
        self._check(self.lib.thc_build_factors(self.ctx, None, None, None, _ptr(Z)), "thc_build_factors")
        return Z

    def mp2_density(self, Z=None):
        """(D_oo, D_vv): the MP2 one-particle density of the amplitudes of core Z (default: the
        current state), App. II."""
        Doo = torch.empty((self.o, self.o), dtype=torch.float64, device="cuda")
        Dvv = torch.empty((self.v, self.v), dtype=torch.float64, device="cuda")
        zp = _ptr(Z, self.nP ** 2, "Z") if Z is not None else None
        self._check(self.lib.thc_mp2_density(self.ctx, zp, _ptr(Doo), _ptr(Dvv)), "thc_mp2_density")
        return Doo, Dvv

    def synth_gamma(self):
        g = C.c_double(0.0)
        self._check(self.lib.thc_synth_gamma(self.ctx, C.byref(g)), "thc_synth_gamma")
        return g.value

    # -- residual -----------------------------------------------------------------------
    def residual(self, Z, t1=None, mask=TERM_ALL, norms=False):
        sig = torch.empty((self.nP, self.nP), dtype=torch.float64, device=Z.device)
        sig1 = torch.zeros((self.o, self.v), dtype=torch.float64, device=Z.device)
        zp = _ptr(Z, self.nP ** 2, "Z")
        tp = _ptr(t1, self.o * self.v, "t1")
        if mask == TERM_ALL and norms:
            nr = (C.c_double * 2)()
            rc = self.lib.thc_residual(self.ctx, zp, tp, _ptr(sig), _ptr(sig1), nr)
            self._check(rc, "thc_residual")
            return sig, sig1, (nr[0], nr[1])
        rc = self.lib.thc_residual_terms(self.ctx, zp, tp, C.c_uint32(mask), _ptr(sig), _ptr(sig1))
        self._check(rc, "thc_residual_terms")
        return sig, sig1

    # -- solver -------------------------------------------------------------------------
    def iterate(self, tol=1e-8, maxit=100, raise_on_notconv=True):
        it = C.c_int(0)
        rn = C.c_double(0.0)
        rc = self.lib.thc_iterate(self.ctx, tol, maxit, C.byref(it), C.byref(rn))
        if rc == THC_ENOTCONV and not raise_on_notconv:
            return it.value, rn.value, False
        self._check(rc, "thc_iterate")
        return it.value, rn.value, True

    def history(self, max_it=1000):
        """(energies, residual norms, seconds) of each iteration of the last iterate() call."""
        e = (C.c_double * max_it)()
        r = (C.c_double * max_it)()
        t = (C.c_double * max_it)()
        n = C.c_int(0)
        self._check(self.lib.thc_history(self.ctx, max_it, e, r, t, C.byref(n)), "thc_history")
        m = min(n.value, max_it)
        return list(e[:m]), list(r[:m]), list(t[:m])

    def iteration_log(self, max_it=1000):
        """One record per iteration of the last iterate() call (a JSON line each, if dumped):
        iteration, energy, its change, residual norm, wall seconds since the call began, and the
        iteration's flags."""
        e, r, t = self.history(max_it)
        f = self.history_flags(max_it)
        out = []
        for k in range(len(e)):
            out.append({"iteration": k + 1, "energy": e[k], "dE": e[k] - e[k - 1] if k else None, "rnorm": r[k],
                        "seconds": t[k], "mixed": bool(f[k] & ITER_MIXED), "restarted": bool(f[k] & ITER_RESTARTED),
                        "diis_dropped": bool(f[k] & ITER_DIIS_DROPPED), "learned": bool(f[k] & ITER_LEARNED)})
        return out

    def history_precision(self, max_it=1000):
        """1 for each iteration of the last iterate() whose residual was mixed precision, else 0."""
        f = (C.c_int * max_it)()
        n = C.c_int(0)
        self._check(self.lib.thc_history_precision(self.ctx, max_it, f, C.byref(n)), "thc_history_precision")
        return list(f[:min(n.value, max_it)])

    def history_flags(self, max_it=1000):
        """THC_ITER_* bits of each iteration of the last iterate() call."""
        f = (C.c_int * max_it)()
        n = C.c_int(0)
        self._check(self.lib.thc_history_flags(self.ctx, max_it, f, C.byref(n)), "thc_history_flags")
        return [f[k] for k in range(min(n.value, max_it))]

    def save_checkpoint(self):
        """The solver state (T^, t1, shift, DIIS subspace, last energy) as a uint8 numpy array."""
        import numpy as np
        n = C.c_size_t(0)
        self._check(self.lib.thc_checkpoint_bytes(self.ctx, C.byref(n)), "thc_checkpoint_bytes")
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self.lib.thc_save_checkpoint(self.ctx, buf.ctypes.data_as(C.c_void_p), n.value),
                    "thc_save_checkpoint")
        return buf

    def load_checkpoint(self, buf):
        import numpy as np
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.thc_load_checkpoint(self.ctx, buf.ctypes.data_as(C.c_void_p), buf.size),
                    "thc_load_checkpoint")

    def energy(self):
        e = C.c_double(0.0)
        self._check(self.lib.thc_energy(self.ctx, C.byref(e)), "thc_energy")
        return e.value

    def get_state(self):
        Z = torch.empty((self.nP, self.nP), dtype=torch.float64, device="cuda")
        t1 = torch.empty((self.o, self.v), dtype=torch.float64, device="cuda")
        self._check(self.lib.thc_get_state(self.ctx, _ptr(Z), _ptr(t1)), "thc_get_state")
        return Z, t1

    def set_state(self, Z, t1=None):
        self._check(self.lib.thc_set_state(self.ctx, _ptr(Z, self.nP ** 2, "Z"), _ptr(t1, self.o * self.v, "t1")),
                    "thc_set_state")

    def memory_bytes(self):
        b = C.c_size_t(0)
        self._check(self.lib.thc_memory_bytes(self.ctx, C.byref(b)), "thc_memory_bytes")
        return b.value

    def plan(self):
        """The residual's blocking and kernel paths (a dict of PlanInfo's fields)."""
        p = PlanInfo()
        self._check(self.lib.thc_plan(self.ctx, C.byref(p)), "thc_plan")
        return {name: getattr(p, name) for name, _ in PlanInfo._fields_}

    # -- learned guess ------------------------------------------------------------------
    def guess_features(self):
        """phi (nP x 10, float32) of the current state (after build_factors: the MP2 guess)."""
        phi = torch.empty((self.nP, GUESS_FEATURES), dtype=torch.float32, device="cuda")
        self._check(self.lib.thc_guess_features(self.ctx, _fptr(phi)), "thc_guess_features")
        return phi

    def guess_apply(self, pred):
        """pred (nP x k, float32): column 0 scales the state, column 1 (if any) shifts the denominators."""
        if pred.dim() != 2 or pred.shape[0] != self.nP:
            raise ValueError("pred must be nP x k")
        self._check(self.lib.thc_guess_apply(self.ctx, _fptr(pred, name="pred"), pred.shape[1]), "thc_guess_apply")

    def set_guess_network(self, net=None):
        """The network (MLP) whose prediction starts the first iterate() after build_factors when the
        context was made with guess=1; None detaches it.  The network must outlive its use."""
        self._guess_net = net
        self._check(self.lib.thc_set_guess_network(self.ctx, net.net if net is not None else None),
                    "thc_set_guess_network")

    def set_shift(self, delta=None):
        self._check(self.lib.thc_set_shift(self.ctx, _ptr(delta, self.nP, "delta")), "thc_set_shift")

    def working(self, residual=False):
        """(T^, sigma^ or None) of the current state in the working basis."""
        Th = torch.empty((self.nP, self.nP), dtype=torch.float64, device="cuda")
        sh = torch.empty_like(Th) if residual else None
        self._check(self.lib.thc_working(self.ctx, _ptr(Th), _ptr(sh)), "thc_working")
        return Th, sh

    def guess_targets(self, Th0, Tstar, sig0):
        c = torch.empty(self.nP, dtype=torch.float64, device="cuda")
        d = torch.empty_like(c)
        n2 = self.nP * self.nP
        self._check(self.lib.thc_guess_targets(self.ctx, _ptr(Th0, n2, "Th0"), _ptr(Tstar, n2, "Tstar"),
                                               _ptr(sig0, n2, "sig0"), _ptr(c), _ptr(d)), "thc_guess_targets")
        return c, d

    # -- profiling ----------------------------------------------------------------------
    def profile(self, enable=True):
        self._check(self.lib.thc_profile(self.ctx, int(enable)), "thc_profile")

    def profile_flops(self):
        """(FP64, FP32, split-BF16) MFMA GEMM flops (2 M N K per product) issued since profile(True)."""
        a, b, c = C.c_double(0.0), C.c_double(0.0), C.c_double(0.0)
        self._check(self.lib.thc_profile_flops(self.ctx, C.byref(a), C.byref(b), C.byref(c)), "thc_profile_flops")
        return a.value, b.value, c.value

    def profile_get(self, name):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(self.lib.thc_profile_get(self.ctx, name.encode(), C.byref(ms), C.byref(n)), "thc_profile_get")
        return ms.value, n.value


class MLP:
    """The learned-guess network (n_in -> width -> width -> n_out, SiLU) on the current GPU."""

    def __init__(self, n_in=GUESS_FEATURES, width=256, n_out=2, seed=1):
        self.lib = load()
        self.n_in, self.width, self.n_out = n_in, width, n_out
        h = C.c_void_p()
        rc = self.lib.thc_mlp_create(n_in, width, n_out, C.c_uint64(seed), _stream(), C.byref(h))
        if rc != 0:
            raise ThcError(rc, "thc_mlp_create failed")
        self.net = h
        n = C.c_int64(0)
        self._check(self.lib.thc_mlp_num_params(self.net, C.byref(n)), "thc_mlp_num_params")
        self.n_params = n.value

    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.thc_mlp_last_error(self.net)
            raise ThcError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "net", None):
            self.lib.thc_mlp_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_norm(self, mu_in, sd_in, mu_out, sd_out):
        arr = lambda a, n: (C.c_float * n)(*[float(x) for x in a])
        self._check(self.lib.thc_mlp_set_norm(self.net, arr(mu_in, self.n_in), arr(sd_in, self.n_in),
                                              arr(mu_out, self.n_out), arr(sd_out, self.n_out)), "thc_mlp_set_norm")

    def fit_norm(self, X, T):
        r = self._rows(X)
        self._check(self.lib.thc_mlp_fit_norm(self.net, _fptr(X, name="X"), _fptr(T, r * self.n_out, "T"), r),
                    "thc_mlp_fit_norm")

    def get_norm(self):
        bufs = [(C.c_float * n)() for n in (self.n_in, self.n_in, self.n_out, self.n_out)]
        self._check(self.lib.thc_mlp_get_norm(self.net, *bufs), "thc_mlp_get_norm")
        return tuple(list(b) for b in bufs)

    def get_params(self):
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._check(self.lib.thc_mlp_get_params(self.net, _fptr(p)), "thc_mlp_get_params")
        return p

    def set_params(self, p):
        self._check(self.lib.thc_mlp_set_params(self.net, _fptr(p, self.n_params, "params")), "thc_mlp_set_params")

    def _rows(self, X):
        if X.dim() != 2 or X.shape[1] != self.n_in:
            raise ValueError("X must be rows x n_in")
        return X.shape[0]

    def forward(self, X):
        r = self._rows(X)
        Y = torch.empty((r, self.n_out), dtype=torch.float32, device="cuda")
        self._check(self.lib.thc_mlp_forward(self.net, _fptr(X, name="X"), r, _fptr(Y)), "thc_mlp_forward")
        return Y

    def forward_noalloc(self, X, Y=None):
        """FP32 forward pass into Y (allocated here if not given) with the library allocating
        nothing: activations in its fixed per-GPU scratch array."""
        r = self._rows(X)
        if Y is None:
            Y = torch.empty((r, self.n_out), dtype=torch.float32, device="cuda")
        self._check(self.lib.thc_mlp_forward_noalloc(self.net, _fptr(X, name="X"), r, _fptr(Y, r * self.n_out, "Y")),
                    "thc_mlp_forward_noalloc")
        return Y

    def infer(self, X):
        r = self._rows(X)
        Y = torch.empty((r, self.n_out), dtype=torch.float32, device="cuda")
        self._check(self.lib.thc_mlp_infer(self.net, _fptr(X, name="X"), r, _fptr(Y)), "thc_mlp_infer")
        return Y

    def loss_grad(self, X, T):
        r = self._rows(X)
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = C.c_float(0.0)
        self._check(self.lib.thc_mlp_loss_grad(self.net, _fptr(X, name="X"), _fptr(T, r * self.n_out, "T"), r,
                                               C.byref(loss), _fptr(g)), "thc_mlp_loss_grad")
        return loss.value, g

    def train_step(self, X, T, lr):
        r = self._rows(X)
        loss = C.c_float(0.0)
        self._check(self.lib.thc_mlp_train_step(self.net, _fptr(X, name="X"), _fptr(T, r * self.n_out, "T"), r,
                                                C.c_float(lr), C.byref(loss)), "thc_mlp_train_step")
        return loss.value
