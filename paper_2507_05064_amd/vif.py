"""Python binding of libvif.so (ctypes): argument marshalling only.

Every computation runs in the HIP library. Arrays are torch tensors on the
GPU (their data_ptr() is passed as a device pointer); the library's stream is
torch's current stream at context creation. There is no CPU fallback: if the
library is not built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvif.so")
_lib = None

MATERN12, MATERN32, GAUSSIAN_ARD, MATERN52 = 0, 1, 2, 3
LIK_GAUSSIAN, LIK_BERNOULLI_LOGIT, LIK_POISSON_LOG, LIK_GAMMA_LOG = 0, 1, 2, 3
FP64, FP32, BF16_IN = 0, 1, 2
KERNELS = {"matern12": MATERN12, "matern32": MATERN32, "gaussian_ard": GAUSSIAN_ARD, "matern52": MATERN52}
LIKELIHOODS = {"gaussian": LIK_GAUSSIAN, "bernoulli_logit": LIK_BERNOULLI_LOGIT, "poisson_log": LIK_POISSON_LOG,
               "gamma_log": LIK_GAMMA_LOG}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16_in": BF16_IN}
PRECONDITIONERS = {"vifdu": 0, "fitc": 1}

STATUS = {0: "VIF_OK", 1: "VIF_E_ARG", 2: "VIF_E_NAN", 3: "VIF_E_NOT_PD", 4: "VIF_E_CG_MAXIT",
          5: "VIF_E_NEWTON", 6: "VIF_E_HIP", 7: "VIF_E_OOM", 8: "VIF_E_STATE"}


class VifError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class vif_config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("m", ctypes.c_int32), ("m_v", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("likelihood", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("tau_m", ctypes.c_double), ("cg_tol", ctypes.c_double), ("cg_maxit", ctypes.c_int32),
                ("newton_maxit", ctypes.c_int32), ("newton_tol", ctypes.c_double), ("lik_param", ctypes.c_double),
                ("max_probes", ctypes.c_int32), ("max_pred", ctypes.c_int64)]


class vif_batch_config(ctypes.Structure):
    _fields_ = [("nprob", ctypes.c_int32), ("d", ctypes.c_int32), ("m", ctypes.c_int32), ("m_v", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("precision", ctypes.c_int32), ("tau_m", ctypes.c_double)]


class vif_laplace_stats(ctypes.Structure):
    _fields_ = [("newton_iters", ctypes.c_int32), ("pcg_iters_total", ctypes.c_int32),
                ("pcg_iters", ctypes.c_int32 * 64), ("halvings", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("psi", ctypes.c_double), ("pcg_rel_residual", ctypes.c_double), ("start_used", ctypes.c_int32),
                ("psi_start", ctypes.c_double), ("levels_fwd", ctypes.c_int32), ("levels_bwd", ctypes.c_int32),
                ("wide_fwd", ctypes.c_int32), ("wide_bwd", ctypes.c_int32)]

    def as_dict(self):
        k = min(self.newton_iters, 64)
        return {"newton_iters": self.newton_iters, "pcg_iters_total": self.pcg_iters_total,
                "pcg_iters": list(self.pcg_iters[:k]), "halvings": self.halvings, "converged": bool(self.converged),
                "psi": self.psi, "pcg_rel_residual": self.pcg_rel_residual, "start_used": bool(self.start_used),
                "psi_start": self.psi_start, "levels_fwd": self.levels_fwd, "levels_bwd": self.levels_bwd,
                "wide_fwd": self.wide_fwd, "wide_bwd": self.wide_bwd}


EXPORTS = ["vif_create", "vif_destroy", "vif_last_error", "vif_select_neighbors", "vif_build_factor", "vif_nll",
           "vif_nll_grad", "vif_export_factor", "vif_set_timing", "vif_timing_stages", "vif_timing_stage_name",
           "vif_get_timing", "vif_laplace_mode", "vif_mlp_num_params", "vif_mlp_workspace_floats",
           "vif_mlp_forward", "vif_mlp_backward", "vif_mlp_adam", "vif_mlp_features", "vif_sample_prior",
           "vif_precond_solve", "vif_set_preconditioner", "vif_batch_create", "vif_batch_destroy", "vif_batch_last_error",
           "vif_batch_nll_grad", "vif_laplace_nll", "vif_laplace_nll_grad", "vif_select_neighbors_pred",
           "vif_predict", "vif_laplace_predict", "vif_mlp_forward_noalloc", "vif_select_inducing"]


def load_library(path: Optional[str] = None):
    """Loads libvif.so; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libvif.so not built ({p}); run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, i32p, dp = ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    lib.vif_create.argtypes = [ctypes.POINTER(vif_config), vp, ctypes.POINTER(vp)]
    lib.vif_create.restype = ctypes.c_int
    lib.vif_destroy.argtypes = [vp]
    lib.vif_destroy.restype = None
    lib.vif_last_error.argtypes = [vp]
    lib.vif_last_error.restype = ctypes.c_char_p
    lib.vif_select_neighbors.argtypes = [vp, vp, vp, dp, i32p]
    lib.vif_select_neighbors.restype = ctypes.c_int
    lib.vif_build_factor.argtypes = [vp, vp, vp, i32p, dp]
    lib.vif_build_factor.restype = ctypes.c_int
    lib.vif_nll.argtypes = [vp, vp, dp]
    lib.vif_nll.restype = ctypes.c_int
    lib.vif_nll_grad.argtypes = [vp, vp, dp, dp]
    lib.vif_nll_grad.restype = ctypes.c_int
    lib.vif_export_factor.argtypes = [vp, vp, vp]
    lib.vif_export_factor.restype = ctypes.c_int
    lib.vif_set_timing.argtypes = [vp, ctypes.c_int]
    lib.vif_set_timing.restype = ctypes.c_int
    lib.vif_timing_stages.argtypes = []
    lib.vif_timing_stages.restype = ctypes.c_int
    lib.vif_timing_stage_name.argtypes = [ctypes.c_int]
    lib.vif_timing_stage_name.restype = ctypes.c_char_p
    lib.vif_get_timing.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.vif_get_timing.restype = ctypes.c_int
    lib.vif_laplace_mode.argtypes = [vp, vp, vp, vp, ctypes.POINTER(vif_laplace_stats)]
    lib.vif_laplace_mode.restype = ctypes.c_int
    lib.vif_precond_solve.argtypes = [vp, vp, vp, vp]
    lib.vif_set_preconditioner.argtypes = [vp, ctypes.c_int32]
    lib.vif_set_preconditioner.restype = ctypes.c_int
    lib.vif_precond_solve.restype = ctypes.c_int
    lib.vif_laplace_nll.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, dp, dp]
    lib.vif_laplace_nll.restype = ctypes.c_int
    lib.vif_laplace_nll_grad.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, dp, dp]
    lib.vif_laplace_nll_grad.restype = ctypes.c_int
    lib.vif_select_inducing.argtypes = [vp, vp, dp, dp, vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int32)]
    lib.vif_select_inducing.restype = ctypes.c_int
    lib.vif_select_neighbors_pred.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.vif_select_neighbors_pred.restype = ctypes.c_int
    lib.vif_predict.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, vp]
    lib.vif_predict.restype = ctypes.c_int
    lib.vif_laplace_predict.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp,
                                        ctypes.POINTER(ctypes.c_int32)]
    lib.vif_laplace_predict.restype = ctypes.c_int
    lib.vif_batch_create.argtypes = [ctypes.POINTER(vif_batch_config), ctypes.POINTER(ctypes.c_int64), vp,
                                     ctypes.POINTER(vp)]
    lib.vif_batch_create.restype = ctypes.c_int
    lib.vif_batch_destroy.argtypes = [vp]
    lib.vif_batch_destroy.restype = None
    lib.vif_batch_last_error.argtypes = [vp]
    lib.vif_batch_last_error.restype = ctypes.c_char_p
    lib.vif_batch_nll_grad.argtypes = [vp, vp, vp, vp, dp, vp, dp, dp]
    lib.vif_batch_nll_grad.restype = ctypes.c_int
    lib.vif_mlp_num_params.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.vif_mlp_num_params.restype = ctypes.c_int64
    lib.vif_mlp_workspace_floats.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    lib.vif_mlp_workspace_floats.restype = ctypes.c_int64
    lib.vif_mlp_forward.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
    lib.vif_mlp_forward.restype = ctypes.c_int
    lib.vif_mlp_forward_noalloc.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    lib.vif_mlp_forward_noalloc.restype = ctypes.c_int
    lib.vif_mlp_backward.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp, vp, dp, vp]
    lib.vif_mlp_backward.restype = ctypes.c_int
    lib.vif_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_int32, vp]
    lib.vif_mlp_adam.restype = ctypes.c_int
    lib.vif_mlp_features.argtypes = [vp, vp, vp]
    lib.vif_mlp_features.restype = ctypes.c_int
    lib.vif_sample_prior.argtypes = [vp, vp, vp, vp]
    lib.vif_sample_prior.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dbl_array(x: Sequence[float]):
    arr = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class VifContext:
    """One vif_ctx (workspace sized for n, d, m, m_v, max_probes probes and
    max_pred prediction points) on torch's current stream."""

    def __init__(self, n: int, d: int, m: int, m_v: int, kernel: str = "matern32",
                 likelihood: str = "gaussian", precision: str = "fp64", tau_m: float = 0.0,
                 cg_tol: float = 1e-6, cg_maxit: int = 1000, newton_maxit: int = 100, newton_tol: float = 1e-9,
                 lik_param: float = 1.0, max_probes: int = 0, max_pred: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the VIF library has no CPU path")
        self.lib = load_library()
        self.cfg = vif_config(n, d, m, m_v, KERNELS[kernel], LIKELIHOODS[likelihood], PRECISIONS[precision],
                              tau_m, cg_tol, cg_maxit, newton_maxit, newton_tol, lik_param, max_probes, max_pred)
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self.lib.vif_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise VifError(rc, "vif_create failed")
        self.h = h
        self.n, self.d, self.m, self.m_v = n, d, m, m_v
        self.n_theta = (d if kernel == "gaussian_ard" else 1) + 2

    def close(self):
        if getattr(self, "h", None):
            self.lib.vif_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != 0:
            raise VifError(rc, self.lib.vif_last_error(self.h).decode())

    def select_neighbors(self, X: torch.Tensor, Z: torch.Tensor, theta) -> torch.Tensor:
        nbr = torch.empty((self.n, self.m_v), dtype=torch.int32, device=X.device)
        th, thp = _dbl_array(theta)
        self._check(self.lib.vif_select_neighbors(self.h, _ptr(X), _ptr(Z) if self.m else None, thp, _ptr(nbr)))
        return nbr

    def build_factor(self, X: torch.Tensor, Z: torch.Tensor, nbr: torch.Tensor, theta):
        th, thp = _dbl_array(theta)
        self._check(self.lib.vif_build_factor(self.h, _ptr(X), _ptr(Z) if self.m else None,
                                              _ptr(nbr) if self.m_v else None, thp))

    def nll(self, y: torch.Tensor) -> float:
        out = ctypes.c_double()
        self._check(self.lib.vif_nll(self.h, _ptr(y), ctypes.byref(out)))
        return out.value

    def nll_grad(self, y: torch.Tensor, n_theta: int):
        out = ctypes.c_double()
        g = np.zeros(n_theta)
        self._check(self.lib.vif_nll_grad(self.h, _ptr(y), ctypes.byref(out),
                                          g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.value, g

    def export_factor(self):
        A = torch.empty((self.n, max(self.m_v, 0)), dtype=torch.float64, device="cuda")
        D = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self._check(self.lib.vif_export_factor(self.h, _ptr(A) if self.m_v else None, _ptr(D)))
        return A, D

    def set_preconditioner(self, kind: str):
        """'vifdu' (default) or 'fitc': the preconditioner of the mode finding and of precond_solve."""
        self._check(self.lib.vif_set_preconditioner(self.h, PRECONDITIONERS[kind]))

    def set_timing(self, enable: bool = True):
        self._check(self.lib.vif_set_timing(self.h, int(enable)))

    def timing(self):
        """{stage name: (total ms, launches)} since the last set_timing."""
        k = self.lib.vif_timing_stages()
        ms = np.zeros(k)
        cnt = np.zeros(k, dtype=np.int64)
        self._check(self.lib.vif_get_timing(self.h, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), k))
        return {self.lib.vif_timing_stage_name(s).decode(): (float(ms[s]), int(cnt[s])) for s in range(k)}

    def laplace_mode(self, y: torch.Tensor, b0: Optional[torch.Tensor] = None, raise_on_error: bool = True):
        """(mode, stats dict, status code). Raises on error unless raise_on_error is False."""
        mode = torch.empty(self.n, dtype=torch.float64, device=y.device)
        st = vif_laplace_stats()
        rc = self.lib.vif_laplace_mode(self.h, _ptr(y), _ptr(b0), _ptr(mode), ctypes.byref(st))
        if raise_on_error:
            self._check(rc)
        return mode, st.as_dict(), rc

    def sample_prior(self, eps1: Optional[torch.Tensor], eps2: torch.Tensor) -> torch.Tensor:
        b = torch.empty(self.n, dtype=torch.float64, device=eps2.device)
        self._check(self.lib.vif_sample_prior(self.h, _ptr(eps1) if self.m else None, _ptr(eps2), _ptr(b)))
        return b

    def laplace_nll(self, y: torch.Tensor, mode: torch.Tensor, eps_n: torch.Tensor, eps_m: Optional[torch.Tensor]):
        """(NLL, log det estimate) with ell = eps_n.shape[0] // 2 SLQ probes."""
        ell = eps_n.shape[0] // 2
        nll, ld = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.vif_laplace_nll(self.h, _ptr(y), _ptr(mode), ell, _ptr(eps_n),
                                             _ptr(eps_m) if self.m else None, ctypes.byref(nll), ctypes.byref(ld)))
        return nll.value, ld.value

    def laplace_nll_grad(self, y: torch.Tensor, mode: torch.Tensor, eps_n: torch.Tensor,
                         eps_m: Optional[torch.Tensor]):
        """(NLL, gradient w.r.t. theta = (sigma1^2, length scale(s), s2)) with
        ell = eps_n.shape[0] // 2 probes."""
        ell = eps_n.shape[0] // 2
        nll = ctypes.c_double()
        g = np.zeros(self.n_theta)
        self._check(self.lib.vif_laplace_nll_grad(self.h, _ptr(y), _ptr(mode), ell, _ptr(eps_n),
                                                  _ptr(eps_m) if self.m else None, ctypes.byref(nll),
                                                  g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return nll.value, g

    def select_inducing(self, X: torch.Tensor, theta, unif=None, Z_init: Optional[torch.Tensor] = None,
                        lloyd_iters: int = 10, return_seed: bool = False):
        """k-means++ inducing points in the transformed space q(s) = s / lambda
        (vif_select_inducing): D^2 seeding with the given uniforms (m values),
        or Lloyd iterations from Z_init."""
        Z = torch.empty((self.m, self.d), dtype=torch.float64, device="cuda")
        th, thp = _dbl_array(theta)
        ua, up = _dbl_array(unif) if unif is not None else (None, None)
        idx = (ctypes.c_int32 * self.m)()
        self._check(self.lib.vif_select_inducing(self.h, _ptr(X), thp, up, _ptr(Z_init), lloyd_iters, _ptr(Z), idx))
        return (Z, np.array(idx[:], dtype=np.int64)) if return_seed else Z

    def select_neighbors_pred(self, Xp: torch.Tensor) -> torch.Tensor:
        nbrp = torch.full((Xp.shape[0], max(self.m_v, 1)), -1, dtype=torch.int32, device="cuda")
        self._check(self.lib.vif_select_neighbors_pred(self.h, _ptr(Xp), Xp.shape[0], _ptr(nbrp)))
        return nbrp

    def predict(self, y: torch.Tensor, Xp: torch.Tensor, nbrp: torch.Tensor, variances: bool = False):
        """Posterior predictive mean at Xp (Prop. 2.1); y = response, or the
        mode for a latent model. With variances=True returns (mean, var), var
        the predictive variances of y^p (Gaussian contexts)."""
        mu = torch.empty(Xp.shape[0], dtype=torch.float64, device="cuda")
        var = torch.empty(Xp.shape[0], dtype=torch.float64, device="cuda") if variances else None
        self._check(self.lib.vif_predict(self.h, _ptr(y), _ptr(Xp), _ptr(nbrp) if self.m_v else None, Xp.shape[0],
                                         _ptr(mu), _ptr(var) if variances else None))
        return (mu, var) if variances else mu

    def laplace_predict(self, y: torch.Tensor, mode: torch.Tensor, Xp: torch.Tensor, nbrp: torch.Tensor,
                        eps_n: torch.Tensor, eps_m: Optional[torch.Tensor]):
        """(omega_p, diag(Omega_p), total CG iterations): the latent predictive
        mean and variances of Prop. 3.1 at the mode, eq. Part2 by simulation (SBPV)
        with ell = eps_n.shape[0] // 2 samples."""
        ell = eps_n.shape[0] // 2
        mu = torch.empty(Xp.shape[0], dtype=torch.float64, device="cuda")
        var = torch.empty(Xp.shape[0], dtype=torch.float64, device="cuda")
        its = ctypes.c_int32()
        self._check(self.lib.vif_laplace_predict(self.h, _ptr(y), _ptr(mode), _ptr(Xp),
                                                 _ptr(nbrp) if self.m_v else None, Xp.shape[0], ell, _ptr(eps_n),
                                                 _ptr(eps_m) if self.m else None, _ptr(mu), _ptr(var),
                                                 ctypes.byref(its)))
        return mu, var, its.value

    def precond_solve(self, W: torch.Tensor, r: torch.Tensor) -> torch.Tensor:
        z = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self._check(self.lib.vif_precond_solve(self.h, _ptr(W), _ptr(r), _ptr(z)))
        return z

    def mlp_features(self, y: torch.Tensor) -> torch.Tensor:
        feat = torch.empty((self.n, MLP_FEATURES), dtype=torch.float32, device=y.device)
        self._check(self.lib.vif_mlp_features(self.h, _ptr(y), _ptr(feat)))
        return feat


MLP_FEATURES = 16


class VifBatch:
    """One vif_batch: many independent Gaussian problems (sizes n_list) that
    share d, m, m_v, the kernel and the precision form."""

    def __init__(self, n_list: Sequence[int], d: int, m: int, m_v: int, kernel: str = "matern32",
                 precision: str = "fp32", tau_m: float = 0.0):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the VIF library has no CPU path")
        self.lib = load_library()
        self.n_list = [int(v) for v in n_list]
        self.nprob = len(self.n_list)
        self.cfg = vif_batch_config(self.nprob, d, m, m_v, KERNELS[kernel], PRECISIONS[precision], tau_m)
        nn = (ctypes.c_int64 * self.nprob)(*self.n_list)
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self.lib.vif_batch_create(ctypes.byref(self.cfg), nn, ctypes.c_void_p(self.stream.cuda_stream),
                                       ctypes.byref(h))
        if rc != 0:
            raise VifError(rc, "vif_batch_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.vif_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nll_grad(self, X: torch.Tensor, Z: torch.Tensor, nbr: torch.Tensor, theta, y: torch.Tensor,
                 grad: bool = True):
        """theta: nprob x 3 (sigma1^2, range, nugget). Returns (nll[nprob],
        grad[nprob, 3] or None) as numpy arrays."""
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(self.nprob, 3))
        nll = np.zeros(self.nprob)
        g = np.zeros((self.nprob, 3)) if grad else None
        dptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rc = self.lib.vif_batch_nll_grad(self.h, _ptr(X), _ptr(Z), _ptr(nbr), dptr(th), _ptr(y), dptr(nll),
                                         dptr(g) if grad else None)
        if rc != 0:
            raise VifError(rc, self.lib.vif_batch_last_error(self.h).decode())
        return nll, g


class VifNLLFunction(torch.autograd.Function):
    """Gaussian VIF negative log-likelihood as a differentiable function of
    theta (a host FP64 tensor: sigma1^2, range or ARD length scales, nugget).
    The forward builds the factor and runs vif_nll_grad, whose adjoint
    (Sec. 2.3, App. A) gives dNLL/dtheta; the backward scales it."""

    @staticmethod
    def forward(fctx, theta, vctx, X, Z, nbr, y):
        th = theta.detach().cpu().double().numpy()
        vctx.build_factor(X, Z, nbr, th)
        nll, g = vctx.nll_grad(y, th.size)
        fctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype))
        return theta.new_tensor(nll)

    @staticmethod
    def backward(fctx, gout):
        (g,) = fctx.saved_tensors
        return gout * g.to(gout.device), None, None, None, None, None


def vif_nll(theta: torch.Tensor, vctx: "VifContext", X: torch.Tensor, Z: Optional[torch.Tensor],
            nbr: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """NLL(theta) with autograd support through the library's adjoint."""
    return VifNLLFunction.apply(theta, vctx, X, Z, nbr, y)


def _mlp_call(rc: int, what: str):
    if rc != 0:
        raise VifError(rc, what)


class WarmStartMLP:
    """The warm-start network's parameters (one flat FP32 device tensor) and
    its Adam state; every computation runs in the library's kernels."""

    def __init__(self, H: int = 128, F: int = MLP_FEATURES, params: Optional[torch.Tensor] = None, seed: int = 0):
        self.lib = load_library()
        self.F, self.H = F, H
        self.P = int(self.lib.vif_mlp_num_params(F, H))
        if params is None:
            g = np.random.default_rng(seed)
            parts = []
            for name, shape in (("W1", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
                                ("b3", (H,)), ("w4", (H,)), ("b4", (1,))):
                if name[0] == "W":
                    parts.append(g.standard_normal(shape).ravel() * np.sqrt(2.0 / shape[0]))
                elif name == "w4":
                    parts.append(g.standard_normal(shape) * np.sqrt(1.0 / shape[0]))
                else:
                    parts.append(np.zeros(int(np.prod(shape))))
            params = torch.as_tensor(np.concatenate(parts).astype(np.float32), device="cuda")
        assert params.numel() == self.P
        self.params = params.contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = None

    def _workspace(self, n: int) -> torch.Tensor:
        need = int(self.lib.vif_mlp_workspace_floats(n, self.F, self.H))
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.float32, device="cuda")
        return self._ws

    def forward(self, X: torch.Tensor, double: bool = False) -> torch.Tensor:
        n = X.shape[0]
        out = torch.empty(n, dtype=torch.float64 if double else torch.float32, device=X.device)
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        _mlp_call(self.lib.vif_mlp_forward(_ptr(self.params), _ptr(X), n, self.F, self.H, _ptr(self._workspace(n)),
                                           None if double else _ptr(out), _ptr(out) if double else None, st),
                  "vif_mlp_forward")
        return out

    def forward_noalloc(self, X: torch.Tensor, double: bool = False) -> torch.Tensor:
        """As forward, through vif_mlp_forward_noalloc (no workspace: the
        library's fixed per-device array holds the hidden layers)."""
        n = X.shape[0]
        out = torch.empty(n, dtype=torch.float64 if double else torch.float32, device=X.device)
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        _mlp_call(self.lib.vif_mlp_forward_noalloc(_ptr(self.params), _ptr(X), n, self.F, self.H,
                                                   None if double else _ptr(out), _ptr(out) if double else None, st),
                  "vif_mlp_forward_noalloc")
        return out

    def loss_grad(self, X: torch.Tensor, target: torch.Tensor):
        n = X.shape[0]
        grad = torch.empty_like(self.params)
        loss = ctypes.c_double()
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        _mlp_call(self.lib.vif_mlp_backward(_ptr(self.params), _ptr(X), _ptr(target), n, self.F, self.H,
                                            _ptr(self._workspace(n)), _ptr(grad), ctypes.byref(loss), st),
                  "vif_mlp_backward")
        return loss.value, grad

    def adam(self, grad: torch.Tensor, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8):
        self.step += 1
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        _mlp_call(self.lib.vif_mlp_adam(_ptr(self.params), _ptr(grad), _ptr(self.m), _ptr(self.v), self.P, lr, beta1,
                                        beta2, eps, self.step, st), "vif_mlp_adam")
