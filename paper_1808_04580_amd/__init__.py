"""Python binding of the NFFT graph-Laplacian library (libnfl.so, gfx950).

Argument marshalling only: every step runs in the HIP library behind the
C-ABI declared in include/nfl.h.  PyTorch supplies device memory and the
stream (the current torch stream of the tensors' device).  If the library is
not built, loading fails loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnfl.so")

NFL_OK = 0
NFL_NOT_CONVERGED = 1
NFL_ERR_ARG = -1
NFL_ERR_ORDER = -2
NFL_ERR_DEGREE = -3
NFL_ERR_HIP = -4
NFL_ERR_OOM = -5
NFL_ERR_UNSUPPORTED = -6

OPT_P = 1
OPT_TILE = 2
OPT_CHUNK = 3
OPT_EPS_B_DEFAULT = 4
OPT_KERNEL = 5
OPT_RESTARTS = 6
KERNELS = {"gaussian": 0, "multiquadric": 1, "inverse_multiquadric": 2, "laplacian_rbf": 3}
OPT_EPS_I = 7
OPT_DETERMINISTIC = 8
OPT_PRECISION = 9

WARM_ZERO = 0
WARM_USER = 1
WARM_MLP = 2
CG_NOALLOC_MAX_N = 1048576

_lib = None

# every exported symbol with its (restype, argtypes)
_i, _i64, _d, _p = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
SIGNATURES = {
    "nfl_create": (_i, [ctypes.POINTER(_p), _i, _p]),
    "nfl_destroy": (_i, [_p]),
    "nfl_set_points": (_i, [_p, _i64, _p]),
    "nfl_set_kernel": (_i, [_p, _d, _i, _i, _d]),
    "nfl_set_kernel_ex": (_i, [_p, _i, _d, _i, _i, _d]),
    "nfl_set_points_frame": (_i, [_p, _i64, _p, _p]),
    "nfl_evaluate": (_i, [_p, _p, _p, _p]),
    "nfl_set_option": (_i, [_p, _i, _d]),
    "nfl_degree": (_i, [_p, _p]),
    "nfl_apply_W": (_i, [_p, _p, _p, _i, _i64]),
    "nfl_apply_Ls": (_i, [_p, _p, _p, _i, _i64]),
    "nfl_apply_A": (_i, [_p, _p, _p, _i, _i64]),
    "nfl_apply_A64": (_i, [_p, _p, _p]),
    "nfl_degree64": (_i, [_p, _p]),
    "nfl_lanczos_smallest": (_i, [_p, _i, _i, _d, _i, _p, _p, _p, _p]),
    "nfl_cg_solve": (_i, [_p, _d, _p, _p, _i, _d, _i, _p, _p]),
    "nfl_cg_solve_noalloc": (_i, [_p, _d, _p, _p, _i, _d, _i, _p, _p]),
    "nfl_nystrom": (_i, [_p, _p, _i64, _i, _i, _i, _p, _p, _p]),
    "nfl_krr_solve": (_i, [_p, _d, _p, _p, _i, _d, _i, _p, _p]),
    "nfl_get_info": (_i, [_p, _p, _p, _p, _p, _p, _p]),
    "nfl_error_estimate": (_i, [_p, _i, ctypes.c_uint64, _p, _p, _p, _p, _p]),
    "nfl_grid_size": (_i64, [_p]),
    "nfl_spread": (_i, [_p, _p, _p]),
    "nfl_convolve": (_i, [_p, _p, _p]),
    "nfl_interp": (_i, [_p, _p, _p]),
    "nfl_get_filter": (_i, [_p, _p, _i64]),
    "nfl_compute_filter": (_i, [_i, _i, _i, _i, _d, _d, _p, _i64]),
    "nfl_compute_filter_ex": (_i, [_i, _i, _i, _i, _i, _d, _d, _d, _p, _i64]),
    "nfl_profile_stages": (_i, [_p, _p, _p, _i, _p]),
    "nfl_window_coefficients": (_i, [_i, _p, _i64]),
    "nfl_mlp_create": (_i, [ctypes.POINTER(_p), _i, ctypes.c_uint64, _p]),
    "nfl_mlp_destroy": (_i, [_p]),
    "nfl_mlp_train_step": (_i, [_p, _p, _p, _p, _i, _i64, ctypes.c_uint64, _d, _p]),
    "nfl_mlp_predict": (_i, [_p, _p, _p, _i, _p]),
    "nfl_mlp_attach": (_i, [_p, _p, _i]),
    "nfl_mlp_save": (_i, [_p, ctypes.c_char_p]),
    "nfl_mlp_load": (_i, [_p, ctypes.c_char_p]),
    "nfl_mlp_get_params": (_i, [_p, _p, _i64]),
    "nfl_mlp_set_params": (_i, [_p, _p, _i64]),
    "nfl_mlp_forward": (_i, [_p, _p, _i64, _p]),
    "nfl_mlp_gradient": (_i, [_p, _p, _p, _i64, _p, _i64, _p]),
    "nfl_direct_rows": (_i, [_p, _d, _p, _p, _i, _p, _p]),
    "nfl_autotune": (_i, [_p, _d, _d, _i, ctypes.c_uint64, ctypes.c_char_p, _p, _p, _p, _p, _p,
                          _p, _p]),
    "nfl_batch_create": (_i, [ctypes.POINTER(_p), _p, _i, _i, _p]),
    "nfl_batch_offsets": (_i, [_p, _p, _i64]),
    "nfl_batch_apply_Ls": (_i, [_p, _p, _p]),
    "nfl_batch_info": (_i, [_p, _p, _p, _p, _p]),
    "nfl_batch_destroy": (_i, [_p]),
    "nfl_strerror": (ctypes.c_char_p, [_i]),
    "nfl_last_error": (ctypes.c_char_p, []),
}


class NFLError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


def lib():
    """Load libnfl.so (built in-tree by paper_1808_04580_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libnfl.so is not built: run python -m paper_1808_04580_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int, where: str, allow_soft: bool = False) -> int:
    if code < 0 or (code > 0 and not allow_soft):
        msg = lib().nfl_last_error().decode(errors="replace")
        raise NFLError(code, where, msg)
    return code


def strerror(code: int) -> str:
    return lib().nfl_strerror(code).decode()


def compute_filter(d: int, N: int, m: int, p: int, eps_B: float, sigma_tilde: float,
                   kind: str = "gaussian", eps_I: float = 0.0) -> np.ndarray:
    """The half-spectrum filter (host FP64, no GPU needed); for kernels other
    than the Gaussian, of the kernel divided by K(0)."""
    count = (N + 1) ** (d - 1) * (N // 2 + 1)
    out = np.empty(count, dtype=np.float64)
    _check(lib().nfl_compute_filter_ex(KERNELS[kind], d, N, m, p, float(eps_B),
                                       float(sigma_tilde), float(eps_I), out.ctypes.data_as(_p),
                                       count),
           "nfl_compute_filter_ex")
    shape = tuple([N + 1] * (d - 1) + [N // 2 + 1])
    return out.reshape(shape)


WIN_NC = 8


def window_coefficients(m: int) -> np.ndarray:
    """(2m, WIN_NC) float32 window polynomial coefficients (host, no GPU)."""
    out = np.empty(2 * m * WIN_NC, dtype=np.float32)
    _check(lib().nfl_window_coefficients(m, out.ctypes.data_as(_p), out.size),
           "nfl_window_coefficients")
    return out.reshape(2 * m, WIN_NC)


def _ptr(t) -> int:
    return t.data_ptr()


class Plan:
    """One graph (vertex set + Gaussian kernel + NFFT parameters) on the
    current device; all work goes on the current torch stream at creation."""

    def __init__(self, d: int, stream=None):
        import torch
        self._torch = torch
        self.d = d
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        h = _p()
        _check(lib().nfl_create(ctypes.byref(h), d, _p(self.stream.cuda_stream)), "nfl_create")
        self._h = h
        self.n = 0

    # -- lifecycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().nfl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- setup --------------------------------------------------------------
    def set_option(self, opt: int, value: float):
        _check(lib().nfl_set_option(self._h, opt, float(value)), "nfl_set_option")
        if opt == OPT_P:
            self._options = dict(getattr(self, "_options", {}), **{opt: value})

    def set_points(self, v):
        torch = self._torch
        v = torch.as_tensor(v, dtype=torch.float32, device=self.device).contiguous()
        if v.dim() == 1:
            v = v[:, None]
        assert v.shape[1] == self.d
        self.n = int(v.shape[0])
        _check(lib().nfl_set_points(self._h, self.n, _ptr(v)), "nfl_set_points")

    def set_kernel(self, sigma: float, N: int, m: int, eps_B: float = 0.0,
                   kind: str = "gaussian"):
        """sigma: the kernel parameter (Gaussian width, or c of the
        (inverse) multiquadric kernel)."""
        _check(lib().nfl_set_kernel_ex(self._h, KERNELS[kind], float(sigma), int(N), int(m),
                                       float(eps_B)), "nfl_set_kernel_ex")
        self._kernel = (float(sigma), int(N), int(m), float(eps_B), kind)
        self._N = int(N)

    def set_points_frame(self, v, src: "Plan"):
        """Target nodes in the frame of plan `src` (nfl_set_points_frame)."""
        torch = self._torch
        v = torch.as_tensor(v, dtype=torch.float32, device=self.device).contiguous()
        _check(lib().nfl_set_points_frame(self._h, v.shape[0], _ptr(v), src._h),
               "nfl_set_points_frame")
        self.n = int(v.shape[0])

    def evaluate(self, x, tgt: "Plan" = None, out=None):
        """y_j = sum_i x_i K(t_j - v_i) at the nodes of target plan tgt
        (default: this plan's own nodes, y = W x + K(0) x)."""
        torch = self._torch
        tgt = self if tgt is None else tgt
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        y = torch.empty(tgt.n, dtype=torch.float32, device=self.device) if out is None else out
        _check(lib().nfl_evaluate(self._h, _ptr(x), tgt._h, _ptr(y)), "nfl_evaluate")
        return y

    def krr_predict(self, alpha, tgt: "Plan"):
        """Kernel ridge regression prediction F(t) = sum_i alpha_i K(t - v_i)
        (Section 6.3) at the target plan's nodes, FP32."""
        return self.evaluate(alpha, tgt)

    def info(self) -> dict:
        vals = [ctypes.c_double() for _ in range(5)]
        p = ctypes.c_int()
        _check(lib().nfl_get_info(self._h, *[ctypes.byref(x) for x in vals], ctypes.byref(p)),
               "nfl_get_info")
        return dict(rho=vals[0].value, sigma_tilde=vals[1].value, dmin=vals[2].value,
                    dmax=vals[3].value, eps_B=vals[4].value, p=p.value)

    def error_estimate(self, samples: int = 4096, seed: int = 0, points=None) -> dict:
        """eta, the sampled ||K_ERR||_inf, eps_est = n ||K_ERR||_inf / ||W||_inf
        and the Lemma's bound (nfl_error_estimate); points: optional (S, d)
        sample points in the scaled coordinates."""
        y = None
        if points is not None:
            y = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, self.d))
            samples = y.shape[0]
        vals = [ctypes.c_double() for _ in range(4)]
        _check(lib().nfl_error_estimate(self._h, int(samples), int(seed),
                                        y.ctypes.data_as(_p) if y is not None else None,
                                        *[ctypes.byref(x) for x in vals]), "nfl_error_estimate")
        return dict(eta=vals[0].value, kerr_inf=vals[1].value, eps_est=vals[2].value,
                    lemma_bound=vals[3].value)

    # -- operators ----------------------------------------------------------
    def degree(self):
        torch = self._torch
        out = torch.empty(self.n, dtype=torch.float32, device=self.device)
        _check(lib().nfl_degree(self._h, _ptr(out)), "nfl_degree")
        return out

    def _apply(self, fn, name, x, out=None):
        torch = self._torch
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        single = x.dim() == 1
        X = x[None, :] if single else x
        assert X.shape[1] == self.n
        Y = torch.empty_like(X) if out is None else out.view(X.shape)
        _check(fn(self._h, _ptr(X), _ptr(Y), int(X.shape[0]), self.n), name)
        return Y[0] if single else Y

    def apply_W(self, x, out=None):
        return self._apply(lib().nfl_apply_W, "nfl_apply_W", x, out)

    def apply_Ls(self, x, out=None):
        return self._apply(lib().nfl_apply_Ls, "nfl_apply_Ls", x, out)

    def apply_A(self, x, out=None):
        return self._apply(lib().nfl_apply_A, "nfl_apply_A", x, out)

    def apply_A64(self, x):
        """A_E x for one FP64 vector in caller order (FP64 throughout on the
        FP64 path, NFL_OPT_PRECISION 64)."""
        torch = self._torch
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        y = torch.empty_like(x)
        _check(lib().nfl_apply_A64(self._h, _ptr(x), _ptr(y)), "nfl_apply_A64")
        return y

    def degree64(self):
        torch = self._torch
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(lib().nfl_degree64(self._h, _ptr(d)), "nfl_degree64")
        return d

    # -- solvers ------------------------------------------------------------
    def lanczos_smallest(self, k: int, tol: float = 1e-8, maxit: int = 300, block: int = 1,
                         vectors: bool = True, restarts: int = 0):
        """k smallest eigenpairs of L_s; restarts > 0 bounds the basis at maxit
        columns and allows that many thick restarts."""
        torch = self._torch
        self.set_option(OPT_RESTARTS, int(restarts))
        ev = np.empty(k, dtype=np.float64)
        V = torch.empty((k, self.n), dtype=torch.float64, device=self.device) if vectors else None
        it = ctypes.c_int()
        res = ctypes.c_double()
        code = _check(lib().nfl_lanczos_smallest(self._h, k, block, float(tol), int(maxit),
                                                 ev.ctypes.data_as(_p),
                                                 _p(_ptr(V)) if V is not None else None,
                                                 ctypes.byref(it), ctypes.byref(res)),
                      "nfl_lanczos_smallest", allow_soft=True)
        return dict(evals=ev, evecs=(V.T if V is not None else None), iters=it.value,
                    max_resid=res.value, converged=(code == NFL_OK))

    def nystrom(self, k: int, L: int = 20, M: int = None, G=None, seed: int = 0,
                vectors: bool = True):
        """Nystrom-Gaussian-NFFT (Alg. nystrom_hybrid): the k largest eigenpairs
        of A_E from the n x L Gaussian matrix G (drawn here from `seed` when not
        given; (n, L) array in caller order)."""
        torch = self._torch
        M = k if M is None else M
        if G is None:
            gen = torch.Generator(device=self.device)
            gen.manual_seed(int(seed))
            Gt = torch.randn((L, self.n), dtype=torch.float64, device=self.device, generator=gen)
        else:
            Gt = torch.as_tensor(G, dtype=torch.float64, device=self.device)
            if Gt.dim() != 2 or Gt.shape[0] != self.n:
                raise ValueError("G must be (n, L)")
            L = Gt.shape[1]
            Gt = Gt.T.contiguous()
        ev = np.empty(k, dtype=np.float64)
        V = torch.empty((k, self.n), dtype=torch.float64, device=self.device) if vectors else None
        mu = ctypes.c_int()
        _check(lib().nfl_nystrom(self._h, _ptr(Gt), self.n, int(L), int(M), int(k),
                                 ev.ctypes.data_as(_p), _p(_ptr(V)) if V is not None else None,
                                 ctypes.byref(mu)), "nfl_nystrom")
        return dict(evals=ev, evals_Ls=1.0 - ev, evecs=(V.T if V is not None else None),
                    m_used=mu.value)

    def cg_solve(self, f, tau: float, tol: float = 1e-6, maxit: int = 1000,
                 warm: int = WARM_ZERO, u0=None, true_residual: bool = True):
        """nfl_cg_solve.  true_residual=False passes no relres pointer: the
        closing product that recomputes the true residual is skipped and
        the result's relres is None."""
        torch = self._torch
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        if u0 is not None:
            u = torch.as_tensor(u0, dtype=torch.float64, device=self.device).clone().contiguous()
            warm = WARM_USER if warm == WARM_ZERO else warm
        else:
            u = torch.zeros_like(f)
        it = ctypes.c_int()
        rel = ctypes.c_double()
        code = _check(lib().nfl_cg_solve(self._h, float(tau), _ptr(f), _ptr(u), int(warm),
                                         float(tol), int(maxit), ctypes.byref(it),
                                         ctypes.byref(rel) if true_residual else None),
                      "nfl_cg_solve", allow_soft=True)
        return dict(u=u, iters=it.value, relres=rel.value if true_residual else None,
                    converged=(code == NFL_OK))

    def cg_solve_noalloc(self, f, u, tau: float, tol: float = 1e-6, maxit: int = 1000,
                         warm: int = WARM_ZERO):
        """nfl_cg_solve_noalloc: the CG solve with its work space in the
        library's static device array (n <= NFL_CG_NOALLOC_MAX_N).  f and u
        are caller-allocated FP64 device tensors of length n (u holds the
        start when warm == WARM_USER; it receives the solution)."""
        it = ctypes.c_int()
        rel = ctypes.c_double()
        code = _check(lib().nfl_cg_solve_noalloc(self._h, float(tau), _ptr(f), _ptr(u), int(warm),
                                                 float(tol), int(maxit), ctypes.byref(it),
                                                 ctypes.byref(rel)), "nfl_cg_solve_noalloc",
                      allow_soft=True)
        return dict(u=u, iters=it.value, relres=rel.value, converged=(code == NFL_OK))

    def krr_solve(self, f, beta: float, tol: float = 1e-6, maxit: int = 1000, alpha0=None):
        """Kernel ridge regression (Section 6.3): alpha = (K + beta I)^{-1} f by
        CG, K the Gram matrix of the plan's kernel (diagonal included)."""
        torch = self._torch
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        if alpha0 is not None:
            a = torch.as_tensor(alpha0, dtype=torch.float64, device=self.device).clone().contiguous()
            warm = WARM_USER
        else:
            a = torch.empty_like(f)
            warm = WARM_ZERO
        it = ctypes.c_int()
        rel = ctypes.c_double()
        code = _check(lib().nfl_krr_solve(self._h, float(beta), _ptr(f), _ptr(a), int(warm),
                                          float(tol), int(maxit), ctypes.byref(it),
                                          ctypes.byref(rel)), "nfl_krr_solve", allow_soft=True)
        return dict(alpha=a, iters=it.value, relres=rel.value, converged=(code == NFL_OK))

    def profile_stages(self, x, nrep: int = 20) -> dict:
        """Average ms per L_s product of: grid clear, spread, convolution, interp, total."""
        torch = self._torch
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        y = torch.empty_like(x)
        out = np.zeros(5)
        _check(lib().nfl_profile_stages(self._h, _ptr(x), _ptr(y), int(nrep),
                                        out.ctypes.data_as(_p)), "nfl_profile_stages")
        return dict(zip(["clear", "spread", "convolve", "interp", "total"], out.tolist()))

    # -- individual steps -----------------------------------------------------
    def grid_size(self) -> int:
        return int(lib().nfl_grid_size(self._h))

    def spread(self, x):
        torch = self._torch
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        g = torch.empty(self.grid_size(), dtype=torch.float32, device=self.device)
        _check(lib().nfl_spread(self._h, _ptr(x), _ptr(g)), "nfl_spread")
        return g

    def convolve(self, g):
        out = self._torch.empty_like(g)
        _check(lib().nfl_convolve(self._h, _ptr(g), _ptr(out)), "nfl_convolve")
        return out

    def interp(self, g):
        torch = self._torch
        f = torch.empty(self.n, dtype=torch.float32, device=self.device)
        _check(lib().nfl_interp(self._h, _ptr(g.contiguous()), _ptr(f)), "nfl_interp")
        return f

    def direct_rows(self, sigma: float, rows, x=None):
        """Exact (W x)_j and d_j on the given caller-order rows (GPU, FP64):
        returns (wx or None, deg) as float64 numpy arrays."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        deg = np.empty(rows.size, dtype=np.float64)
        wx = np.empty(rows.size, dtype=np.float64) if x is not None else None
        xp = _ptr(x.contiguous()) if x is not None else None
        _check(lib().nfl_direct_rows(self._h, float(sigma), xp, rows.ctypes.data_as(_p), rows.size,
                                     wx.ctypes.data_as(_p) if wx is not None else None,
                                     deg.ctypes.data_as(_p)), "nfl_direct_rows")
        return wx, deg

    def autotune(self, sigma: float, target: float = 1e-5, rows: int = 256, seed: int = 1,
                 cache: str | None = None) -> dict:
        """Search (N, m, eps_B, tile) for this plan (nfl_autotune); the plan is
        left set to the result."""
        N, m, tile, cached = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        eps, err, ms = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        code = _check(lib().nfl_autotune(self._h, float(sigma), float(target), int(rows), int(seed),
                                         cache.encode() if cache else None, ctypes.byref(N),
                                         ctypes.byref(m), ctypes.byref(eps), ctypes.byref(tile),
                                         ctypes.byref(err), ctypes.byref(ms), ctypes.byref(cached)),
                      "nfl_autotune", allow_soft=True)
        return {"N": N.value, "m": m.value, "eps_B": eps.value, "tile": tile.value,
                "err": err.value, "ms": ms.value, "cached": bool(cached.value),
                "reached": code == NFL_OK}

    def filter(self) -> np.ndarray:
        N = self._N
        count = (N + 1) ** (self.d - 1) * (N // 2 + 1)
        out = np.empty(count, dtype=np.float64)
        _check(lib().nfl_get_filter(self._h, out.ctypes.data_as(_p), count), "nfl_get_filter")
        return out


def target_plan(points, src: "Plan", stream=None):
    """A plan of target nodes in the frame of `src`, with src's kernel and NFFT
    parameters (for Plan.evaluate / Plan.krr_predict)."""
    import torch
    v = torch.as_tensor(points)
    d = 1 if v.dim() == 1 else int(v.shape[1])
    T = Plan(d, stream)
    for opt, val in getattr(src, "_options", {}).items():
        T.set_option(opt, val)
    T.set_points_frame(v.reshape(-1, d), src)
    sigma, N, m, eps_B, kind = src._kernel
    T.set_kernel(sigma, N, m, eps_B, kind=kind)
    return T


def plan(points, sigma: float, N: int, m: int, eps_B: float = 0.0, stream=None,
         kind: str = "gaussian", **options):
    """Create, fill and return a Plan for float32 points (n, d) on the GPU."""
    import torch
    v = torch.as_tensor(points)
    d = 1 if v.dim() == 1 else int(v.shape[1])
    P = Plan(d, stream)
    for k, val in options.items():
        P.set_option({"p": OPT_P, "tile": OPT_TILE, "chunk": OPT_CHUNK, "kernel": OPT_KERNEL,
                      "eps_I": OPT_EPS_I, "deterministic": OPT_DETERMINISTIC,
                      "precision": OPT_PRECISION}[k],
                     val)
    P.set_points(v)
    P.set_kernel(sigma, N, m, eps_B, kind=kind)
    return P


class Batch:
    """Several d = 3 plans, nvec vectors each, applied together by one HIP
    graph launch (nfl_batch_*).  The plans must stay alive and unchanged
    while the batch exists; x and y use the packed layout of
    nfl_batch_offsets: plan g's block is x[nvec*off[g] : nvec*off[g+1]],
    vector j of it x[nvec*off[g] + j*n_g : ... + n_g]."""

    def __init__(self, plans, nvec: int, stream=None):
        import torch
        self._torch = torch
        self.plans = list(plans)
        self.nvec = int(nvec)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        hs = (_p * len(self.plans))(*[P._h for P in self.plans])
        h = _p()
        _check(lib().nfl_batch_create(ctypes.byref(h), hs, len(self.plans), self.nvec,
                                      _p(self.stream.cuda_stream)), "nfl_batch_create")
        self._h = h
        off = np.zeros(len(self.plans) + 1, dtype=np.int64)
        _check(lib().nfl_batch_offsets(self._h, off.ctypes.data_as(_p), off.size), "nfl_batch_offsets")
        self.offsets = off
        self.total_n = int(off[-1])

    def close(self):
        if getattr(self, "_h", None):
            lib().nfl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        tn, nb = ctypes.c_int64(), ctypes.c_int64()
        nj, nk = ctypes.c_int(), ctypes.c_int()
        _check(lib().nfl_batch_info(self._h, ctypes.byref(tn), ctypes.byref(nj), ctypes.byref(nk),
                                    ctypes.byref(nb)), "nfl_batch_info")
        return {"total_n": tn.value, "jobs": nj.value, "kernels": nk.value,
                "arena_bytes": nb.value}

    def pack(self, blocks):
        """Packed float32 device vector from per-plan (nvec, n_g) blocks."""
        t = self._torch
        parts = [t.as_tensor(b, dtype=t.float32, device=self.stream.device).reshape(-1)
                 for b in blocks]
        return t.cat(parts).contiguous()

    def unpack(self, y):
        """Per-plan (nvec, n_g) views of a packed vector."""
        return [y[self.nvec * int(a):self.nvec * int(b)].view(self.nvec, int(b - a))
                for a, b in zip(self.offsets[:-1], self.offsets[1:])]

    def apply_Ls(self, x, out=None):
        t = self._torch
        x = x.contiguous()
        if x.dtype != t.float32 or x.numel() != self.nvec * self.total_n:
            raise ValueError("x must be float32 with nvec * total_n elements")
        y = out if out is not None else t.empty_like(x)
        _check(lib().nfl_batch_apply_Ls(self._h, _ptr(x), _ptr(y)), "nfl_batch_apply_Ls")
        return y


MLP_NP = 9473


class WarmStart:
    """The pointwise warm-start network (BF16 matrix-core MLP) for cg_solve."""

    def __init__(self, n_classes: int = 3, seed: int = 0, stream=None):
        import torch
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        h = _p()
        _check(lib().nfl_mlp_create(ctypes.byref(h), n_classes, seed, _p(self.stream.cuda_stream)),
               "nfl_mlp_create")
        self._h = h
        self.n_classes = n_classes

    def close(self):
        if getattr(self, "_h", None):
            lib().nfl_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(MLP_NP, dtype=np.float32)
        _check(lib().nfl_mlp_get_params(self._h, out.ctypes.data_as(_p), MLP_NP), "nfl_mlp_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        _check(lib().nfl_mlp_set_params(self._h, p.ctypes.data_as(_p), p.size), "nfl_mlp_set_params")

    def forward(self, feat):
        torch = self._torch
        f = torch.as_tensor(feat, dtype=torch.float32, device=self.device).contiguous()
        out = torch.empty(f.shape[0], dtype=torch.float32, device=self.device)
        _check(lib().nfl_mlp_forward(self._h, _ptr(f), int(f.shape[0]), _ptr(out)), "nfl_mlp_forward")
        return out

    def gradient(self, feat, target):
        torch = self._torch
        f = torch.as_tensor(feat, dtype=torch.float32, device=self.device).contiguous()
        t = torch.as_tensor(target, dtype=torch.float32, device=self.device).contiguous()
        g = np.empty(MLP_NP, dtype=np.float32)
        loss = ctypes.c_double()
        _check(lib().nfl_mlp_gradient(self._h, _ptr(f), _ptr(t), int(f.shape[0]),
                                      g.ctypes.data_as(_p), MLP_NP, ctypes.byref(loss)),
               "nfl_mlp_gradient")
        return loss.value, g

    def train_step(self, plan: "Plan", f, u, cls: int, nsample: int, seed: int, lr: float) -> float:
        torch = self._torch
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        u = torch.as_tensor(u, dtype=torch.float64, device=self.device).contiguous()
        loss = ctypes.c_double()
        _check(lib().nfl_mlp_train_step(self._h, plan._h, _ptr(f), _ptr(u), int(cls), int(nsample),
                                        int(seed), float(lr), ctypes.byref(loss)),
               "nfl_mlp_train_step")
        return loss.value

    def predict(self, plan: "Plan", f, cls: int):
        torch = self._torch
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        u = torch.empty_like(f)
        _check(lib().nfl_mlp_predict(self._h, plan._h, _ptr(f), int(cls), _ptr(u)), "nfl_mlp_predict")
        return u

    def attach(self, plan: "Plan", cls: int):
        """Use this network for plan.cg_solve(..., warm=WARM_MLP); the plan keeps
        a reference to it, and closing the network detaches it from the plan."""
        _check(lib().nfl_mlp_attach(plan._h, self._h, int(cls)), "nfl_mlp_attach")
        plan._warm = self

    def save(self, path: str):
        _check(lib().nfl_mlp_save(self._h, path.encode()), "nfl_mlp_save")

    def load(self, path: str):
        _check(lib().nfl_mlp_load(self._h, path.encode()), "nfl_mlp_load")
