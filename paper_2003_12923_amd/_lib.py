"""ctypes binding of libesmp2 (names follow include/esmp2.h)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libesmp2.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2003_12923_amd.build` (or __graft_entry__.build())")
lib = C.CDLL(LIB_PATH)

(ESMP2_OK, ESMP2_INVALID_ARG, ESMP2_BAD_ORDER, ESMP2_NOT_SPD, ESMP2_NOT_CONVERGED,
 ESMP2_OOM, ESMP2_HIP_ERROR, ESMP2_UNSUPPORTED) = range(8)
ESMP2_FP64, ESMP2_FP32, ESMP2_BF16 = 0, 1, 2
SYLVESTER_VARIANTS = 6
ESMP2_BASIS_TOP, ESMP2_BASIS_SEMICANONICAL = 0, 1
STATUS_NAMES = ["OK", "INVALID_ARG", "BAD_ORDER", "NOT_SPD", "NOT_CONVERGED", "OOM",
                "HIP_ERROR", "UNSUPPORTED"]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int),
                ("x0", C.c_void_p), ("x_out", C.c_void_p), ("resid_hist", C.c_void_p),
                ("inner_tol", C.c_double), ("basis", C.c_int)]


class SolveResult(C.Structure):
    _fields_ = [("e2", C.c_double), ("e2_dl", C.c_double), ("e2_s", C.c_double),
                ("e0", C.c_double), ("rel_resid", C.c_double), ("iterations", C.c_int),
                ("outer", C.c_int), ("status", C.c_int)]


_H = C.c_void_p
_sig = {
    "esmp2_create": ([C.POINTER(_H), C.c_int, C.c_void_p], C.c_int),
    "esmp2_destroy": ([_H], C.c_int),
    "esmp2_set_problem": ([_H, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_int, C.c_int], C.c_int),
    "esmp2_rotate_top": ([_H, C.c_void_p], C.c_int),
    "esmp2_space": ([_H, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "esmp2_build_rhs": ([_H, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "esmp2_sigma": ([_H, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "esmp2_solve": ([_H, C.POINTER(SolveOpts), C.POINTER(SolveResult)], C.c_int),
    "esmp2_gemm_f64": ([_H, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "esmp2_profile": ([_H, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
    "esmp2_solve_batch": ([C.POINTER(_H), C.c_int, C.POINTER(SolveOpts), C.POINTER(SolveResult), C.c_int],
                          C.c_int),
    "esmp2_fock_from_core": ([_H, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
                             C.c_int),
    "esmp2_fock_from_core_noalloc": ([_H, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p], C.c_int),
    "esmp2_set_problem_top": ([_H, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int],
                              C.c_int),
    "esmp2_gradient": ([_H, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "esmp2_autotune": ([_H, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)], C.c_int),
    "esmp2_set_sylvester_variant": ([_H, C.c_int, C.c_int], C.c_int),
    "esmp2_sigma_basis": ([_H, C.c_void_p, C.c_void_p, C.c_int, C.c_int], C.c_int),
    "esmp2_export_determinants": ([_H, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64], C.c_int),
    "esmp2_last_error": ([_H], C.c_char_p),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res


class Esmp2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")
        self.status = status


def _ptr(t):
    """Device address of a tensor; the C ABI takes dense row-major arrays, so a
    strided view is refused rather than read in the wrong order."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor arguments must be contiguous (row-major)")
    return C.c_void_p(t.data_ptr())


class Handle:
    """One library handle bound to a device and a torch stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self.device = device
        if stream == "new":
            stream = torch.cuda.Stream(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.h = _H()
        st = lib.esmp2_create(C.byref(self.h), device, C.c_void_p(stream.cuda_stream))
        if st != ESMP2_OK:
            raise Esmp2Error(st, "esmp2_create failed")

    def _check(self, st, allow=()):
        if st != ESMP2_OK and st not in allow:
            raise Esmp2Error(st, lib.esmp2_last_error(self.h).decode())
        return st

    def close(self):
        if self.h:
            lib.esmp2_destroy(self.h)
            self.h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_problem(self, F, B, Cm, n_occ, n_vir, n_aux, spin=0, n_top=1):
        self._n_occ = n_occ
        return self._check(lib.esmp2_set_problem(self.h, n_occ, n_vir, n_aux, _ptr(F), _ptr(B),
                                                 _ptr(Cm), spin, n_top))

    def set_problem_top(self, Ft, Bt, lam, n_occ, n_vir, n_aux, spin=0):
        self._n_occ = n_occ
        return self._check(lib.esmp2_set_problem_top(self.h, n_occ, n_vir, n_aux, _ptr(Ft), _ptr(Bt), _ptr(lam),
                                                     spin))

    def gradient(self, x, dF=None, dB=None):
        """dE2/dF~ into dF (N x N) and dE2/dB~ into dB (n_aux x N x N), either may be None."""
        return self._check(lib.esmp2_gradient(self.h, _ptr(x), _ptr(dF), _ptr(dB)))

    def rotate_top(self, lam_out=True):
        import numpy as np
        if not lam_out:
            self._check(lib.esmp2_rotate_top(self.h, None))
            return None
        lam = np.zeros(self._n_occ, dtype=np.float64)
        self._check(lib.esmp2_rotate_top(self.h, lam.ctypes.data_as(C.c_void_p)))
        return lam

    def space(self):
        n = C.c_int64()
        offs = (C.c_int64 * 8)()
        self._check(lib.esmp2_space(self.h, C.byref(n), offs))
        return n.value, list(offs)

    def build_rhs(self, b_out=None, e2_s=True):
        """Returns (E0, E2_S).  With e2_s=False the S-triple energy is not waited
        for (it is computed beside the solve and reported in its result): (E0, None)."""
        e0, e2s = C.c_double(), C.c_double()
        self._check(lib.esmp2_build_rhs(self.h, _ptr(b_out), C.byref(e0), C.byref(e2s) if e2_s else None))
        return e0.value, (e2s.value if e2_s else None)

    def sigma(self, x, y, precision=ESMP2_FP64):
        return self._check(lib.esmp2_sigma(self.h, _ptr(x), _ptr(y), precision))

    def sigma_basis(self, x, y, precision=ESMP2_FP64, basis=ESMP2_BASIS_TOP):
        return self._check(lib.esmp2_sigma_basis(self.h, _ptr(x), _ptr(y), precision, basis))

    def export_determinants(self, x, coeff, keys):
        """Determinant coefficients and keys of the TOP-basis amplitudes x (device tensors)."""
        return self._check(lib.esmp2_export_determinants(self.h, _ptr(x), _ptr(coeff), _ptr(keys), coeff.numel()))

    def solve(self, tol=1e-8, max_iter=200, precision=ESMP2_FP64, x0=None, x_out=None,
              history=False, inner_tol=0.0, basis=ESMP2_BASIS_TOP, allow=(ESMP2_NOT_CONVERGED,)):
        import numpy as np
        hist = np.zeros(max_iter, dtype=np.float64) if history else None
        o = SolveOpts(tol, max_iter, precision, None if x0 is None else x0.data_ptr(),
                      None if x_out is None else x_out.data_ptr(),
                      None if hist is None else hist.ctypes.data, inner_tol, basis)
        r = SolveResult()
        self._check(lib.esmp2_solve(self.h, C.byref(o), C.byref(r)), allow=allow)
        out = {k: getattr(r, k) for k, _ in SolveResult._fields_}
        if hist is not None:
            out["history"] = hist[: r.iterations].copy()
        return out

    def profile(self, enable=True):
        """{precision: (ms, launches)} of the Sylvester kernel since the last call."""
        ms, n = (C.c_double * 3)(), (C.c_int64 * 3)()
        self._check(lib.esmp2_profile(self.h, 1 if enable else 0, ms, n))
        return {ESMP2_FP64: (ms[0], n[0]), ESMP2_FP32: (ms[1], n[1]), ESMP2_BF16: (ms[2], n[2])}

    def autotune(self, precision=ESMP2_FP64, reps=5):
        """Time every Sylvester variant; returns (fastest, [ms per launch or -1])."""
        v = C.c_int(-1)
        ms = (C.c_double * SYLVESTER_VARIANTS)()
        self._check(lib.esmp2_autotune(self.h, precision, reps, C.byref(v), ms))
        return v.value, list(ms)

    def set_sylvester_variant(self, precision, variant):
        return self._check(lib.esmp2_set_sylvester_variant(self.h, precision, variant))

    def fock_from_core(self, hcore, B, Cm, n_occ, n_vir, n_aux, F_out):
        return self._check(lib.esmp2_fock_from_core(self.h, n_occ, n_vir, n_aux, _ptr(hcore), _ptr(B), _ptr(Cm),
                                                    _ptr(F_out)))

    def fock_from_core_noalloc(self, hcore, B, Cm, n_occ, n_vir, n_aux, F_out):
        return self._check(lib.esmp2_fock_from_core_noalloc(self.h, n_occ, n_vir, n_aux, _ptr(hcore), _ptr(B),
                                                            _ptr(Cm), _ptr(F_out)))

    def gemm_f64(self, A, B, Cm):
        m, k = A.shape
        n = B.shape[1]
        return self._check(lib.esmp2_gemm_f64(self.h, m, n, k, _ptr(A), _ptr(B), _ptr(Cm)))

    # convenience: bind a synthetic problem held in numpy arrays
    def load(self, prob, spin=0, n_top=1):
        import torch
        dev = f"cuda:{self.device}"
        self._F = torch.from_numpy(prob.F).to(dev)
        self._B = torch.from_numpy(prob.B).to(dev)
        self._C = torch.from_numpy(prob.C).to(dev)
        self._n_occ = prob.n_occ
        self.n_top = n_top
        self.set_problem(self._F, self._B, self._C, prob.n_occ, prob.n_vir, prob.n_aux, spin=spin, n_top=n_top)
        return self

    def load_threshold(self, prob, eta, spin=0):
        """Bind prob with the large TOPs chosen by a singular-value threshold
        (paper Sec. II.C): one rotation with one large TOP gives the singular
        values of C, then the problem is bound again with
        n_top = large_top_count(lambda, eta) (the amplitude layout depends on it).
        The chosen count is in self.n_top."""
        self.load(prob, spin=spin, n_top=1)
        k = large_top_count(self.rotate_top(), eta)
        if k != 1:
            self.load(prob, spin=spin, n_top=k)
        return self


def large_top_count(lam, eta):
    """Number of transition-orbital pairs treated as large under the threshold
    eta on the singular values of C (paper Sec. II.C): those with lambda >= eta,
    at least one (the dominant pair is always large)."""
    return max(1, sum(1 for v in lam if v >= eta))


def solve_batch(handles, tol=1e-8, max_iter=300, precision=ESMP2_FP64, basis=ESMP2_BASIS_TOP, inner_tol=0.0,
                n_threads=8):
    """Rotation, right-hand side, solve and E2 for every handle (each bound to a
    problem and to its own stream); returns one result dict per handle."""
    n = len(handles)
    arr = (_H * n)(*[hd.h for hd in handles])
    o = SolveOpts(tol, max_iter, precision, None, None, None, inner_tol, basis)
    res = (SolveResult * n)()
    st = lib.esmp2_solve_batch(arr, n, C.byref(o), res, n_threads)
    out = [{k: getattr(r, k) for k, _ in SolveResult._fields_} for r in res]
    if st not in (ESMP2_OK, ESMP2_NOT_CONVERGED):
        bad = next((i for i, r in enumerate(out) if r["status"] not in (ESMP2_OK, ESMP2_NOT_CONVERGED)), 0)
        raise Esmp2Error(st, lib.esmp2_last_error(handles[bad].h).decode())
    return out
