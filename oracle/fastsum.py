"""Oracle B: the trigonometric kernel approximation of Section 3 in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. nfft_fastsum approximates (W~ x)_j = sum_i x_i K(v_j - v_i), W~ = W + K(0) I,
by replacing K with a trigonometric polynomial K_RF whose coefficients come
from the regularised kernel K_R (eq. K_RF, eq. b_l::K_RF).  The NFFTs inside the
algorithm only approximate the two nonequispaced sums; this module evaluates
those sums *exactly* by direct nonequispaced DFTs, so that

    HIP path  vs  this module   = window / FFT / FP32 error of the NFFT,
    this module vs direct sums  = kernel-approximation error (N, eps_B, p).

Readings of the paper taken here (listed with the rest in the design notes):
* eq. b_l::K_RF prints the normalisation 1/N; for d > 1 the trapezoidal rule
  needs 1/N^d so that K_RF interpolates K_R at the nodes j/N.  1/N^d is used.
* I_N = {-N/2, ..., N/2-1}^d is not symmetric, so the sum of Alg. nfft_fastsum
  is complex in general; its real part is taken.  That is the same as
  splitting each Nyquist coefficient evenly between +l and -l, and it makes
  the operator real and symmetric.
* K_R (the regularisation ansatz after Section 3's ansatz figure): K inside
  radius 1/2 - eps_B, a polynomial T_B(r) on (1/2 - eps_B, 1/2], the constant
  T_B(1/2) outside.  T_B is the two-point Taylor (Hermite) interpolant of
  degree 2p-1 that matches K and its first p-1 radial derivatives at
  r0 = 1/2 - eps_B, takes the value K(1/2) at r = 1/2 and has vanishing
  derivatives 1..p-1 there, so K_R is p-1 times continuously differentiable.
* Nodes are shifted to their bounding-box midpoint and always scaled so that
  the largest norm is exactly 1/4 - eps_B/2 (Alg. nfft_normalized_matvec,
  steps 1-2); sigma becomes rho * sigma.  W itself does not change.
* Other radial kernels of eq. W_general (multiquadric (r^2 + c^2)^{1/2},
  inverse multiquadric (r^2 + c^2)^{-1/2}): c is a length like sigma, so in
  the scaled coordinates it becomes rho * c and, both kernels being
  homogeneous in (r, c), the sums come out multiplied by rho (multiquadric)
  or 1/rho (inverse multiquadric); they are divided by that factor
  afterwards.  (Alg. nfft_normalized_matvec prints c/rho and the reverse
  factors, which contradicts this homogeneity; the direct sums in the
  original coordinates decide, see the pins.)
"""
from __future__ import annotations

import math

import numpy as np


# ---- Alg. nfft_normalized_matvec, steps 1-2: shift and scale ---------------

def scaling(v, eps_B: float):
    """Return (centre, rho, scaled nodes) with max ||rho (v - c)|| = 1/4 - eps_B/2."""
    V = np.asarray(v, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    c = 0.5 * (V.min(axis=0) + V.max(axis=0))
    R = np.sqrt(((V - c) ** 2).sum(axis=1)).max()
    rho = (0.25 - 0.5 * eps_B) / R if R > 0 else 1.0
    return c, rho, (V - c) * rho


# ---- the Gaussian and its radial derivatives --------------------------------

def gaussian(r, sigma):
    r = np.asarray(r, dtype=np.float64)
    return np.exp(-(r / sigma) ** 2)


def gaussian_radial_derivs(r0: float, sigma: float, p: int):
    """[K(r0), K'(r0), ..., K^{(p-1)}(r0)] for K(r) = exp(-r^2/sigma^2).

    d^k/dr^k exp(-(r/s)^2) = (-1/s)^k H_k(r/s) exp(-(r/s)^2), with the
    physicists' Hermite polynomials H_0 = 1, H_1 = 2x, H_{k+1} = 2x H_k - 2k H_{k-1}.
    """
    x = r0 / sigma
    e = math.exp(-x * x)
    H = [1.0, 2.0 * x]
    for k in range(1, p):
        H.append(2.0 * x * H[k] - 2.0 * k * H[k - 1])
    return [((-1.0 / sigma) ** k) * H[k] * e for k in range(p)]


def two_point_taylor(a: float, b: float, A, B):
    """Coefficients c_q (q < 2p) of T(r) = sum_q c_q t^q, t = (r - a)/(b - a),
    with T^{(k)}(a) = A[k] and T^{(k)}(b) = B[k] for k < p (derivatives in r).

    Written as the 2p x 2p linear system of the Hermite conditions and solved
    with numpy (a library primitive)."""
    p = len(A)
    h = b - a
    nq = 2 * p
    M = np.zeros((nq, nq))
    rhs = np.zeros(nq)
    for k in range(p):
        # k-th t-derivative of t^q at t = 0 is k! if q == k
        M[k, k] = math.factorial(k)
        rhs[k] = A[k] * h ** k
        # at t = 1: q!/(q-k)!
        for q in range(k, nq):
            M[p + k, q] = math.factorial(q) / math.factorial(q - k)
        rhs[p + k] = B[k] * h ** k
    return np.linalg.solve(M, rhs)


# ---- other radial kernels of eq. W_general -----------------------------------

KINDS = ("gaussian", "multiquadric", "inverse_multiquadric", "laplacian_rbf")
_ALPHA = {"multiquadric": 0.5, "inverse_multiquadric": -0.5}


def radial_kernel(kind: str, param: float):
    """K as a function of r = ||y||: exp(-r^2/s^2) (param = s), or
    (r^2 + c^2)^alpha with alpha = 1/2 (multiquadric) or -1/2 (inverse
    multiquadric), param = c."""
    if kind == "gaussian":
        return lambda r: gaussian(r, param)
    if kind == "laplacian_rbf":
        return lambda r: np.exp(-np.asarray(r, dtype=np.float64) / param)
    a = _ALPHA[kind]
    return lambda r: (np.asarray(r, dtype=np.float64) ** 2 + param * param) ** a


def power_radial_derivs(r0: float, c: float, alpha: float, p: int):
    """[K(r0), ..., K^{(p-1)}(r0)] for K(r) = (r^2 + c^2)^alpha.

    With u0 = r0^2 + c^2 and t(h) = (2 r0 h + h^2)/u0,
    K(r0 + h) = u0^alpha (1 + t)^alpha = u0^alpha sum_j binom(alpha, j) t^j,
    and t^j = h^j (2 r0 + h)^j / u0^j contributes binom(j, k - j) (2 r0)^(2j-k)
    / u0^j to the coefficient of h^k (k/2 <= j <= k); K^{(k)}(r0) is k! times
    that coefficient."""
    u0 = r0 * r0 + c * c

    def gbinom(a, j):
        out = 1.0
        for i in range(j):
            out *= (a - i) / (i + 1)
        return out

    out = []
    for k in range(p):
        acc = 0.0
        for j in range((k + 1) // 2, k + 1):
            acc += gbinom(alpha, j) * math.comb(j, k - j) * (2.0 * r0) ** (2 * j - k) / u0 ** j
        out.append(math.factorial(k) * u0 ** alpha * acc)
    return out


def radial_derivs(kind: str, r0: float, param: float, p: int):
    if kind == "gaussian":
        return gaussian_radial_derivs(r0, param, p)
    if kind == "laplacian_rbf":
        # d^k/dr^k exp(-r/s) = (-1/s)^k exp(-r/s)
        return [(-1.0 / param) ** k * math.exp(-r0 / param) for k in range(p)]
    return power_radial_derivs(r0, param, _ALPHA[kind], p)


def scaled_param(kind: str, param: float, rho: float) -> float:
    """The kernel parameter in the scaled coordinates (a length: times rho)."""
    return param * rho


def output_scale(kind: str, rho: float) -> float:
    """K(y; param) = output_scale * K(rho y; rho param) (homogeneity)."""
    return {"gaussian": 1.0, "multiquadric": 1.0 / rho, "inverse_multiquadric": rho,
            "laplacian_rbf": 1.0}[kind]


class RegKernel:
    """K_R of the regularisation ansatz, as a radial function (Gaussian by
    default; `kind` selects another kernel of eq. W_general, `sigma` is then
    its parameter c).  With eps_I > 0 (the Laplacian RBF kernel, not smooth at
    0) K_R is also replaced near the origin: on r <= eps_I by the even
    polynomial T_I of degree 2p - 1 that matches K and its first p - 1 radial
    derivatives at r = +-eps_I (two-point Taylor on [-eps_I, eps_I] of the even
    extension of K), the near-origin regularisation the paper takes from its
    reference on fast summation with singular kernels."""

    def __init__(self, sigma: float, eps_B: float, p: int, kind: str = "gaussian",
                 eps_I: float = 0.0):
        self.sigma, self.eps_B, self.p = float(sigma), float(eps_B), int(p)
        self.kind = kind
        self.eps_I = float(eps_I)
        self.K = radial_kernel(kind, self.sigma)
        self.r0 = 0.5 - self.eps_B
        self.k_half = float(self.K(0.5))
        if self.eps_B > 0:
            A = radial_derivs(kind, self.r0, self.sigma, self.p)
            B = [self.k_half] + [0.0] * (self.p - 1)
            self.coef = two_point_taylor(self.r0, 0.5, A, B)
        else:
            self.coef = None
        if self.eps_I > 0:
            D = radial_derivs(kind, self.eps_I, self.sigma, self.p)
            Dm = [(-1.0) ** k * D[k] for k in range(self.p)]   # even extension at -eps_I
            self.coef_I = two_point_taylor(-self.eps_I, self.eps_I, Dm, D)
        else:
            self.coef_I = None

    def T_I(self, r):
        t = (np.asarray(r, dtype=np.float64) + self.eps_I) / (2.0 * self.eps_I)
        return np.polynomial.polynomial.polyval(t, self.coef_I)

    def near(self, r):
        """K - K_R on r <= eps_I (the near-field correction), 0 elsewhere."""
        r = np.asarray(r, dtype=np.float64)
        if self.coef_I is None:
            return np.zeros_like(r)
        return np.where(r <= self.eps_I, self.K(r) - self.T_I(np.minimum(r, self.eps_I)), 0.0)

    def T_B(self, r):
        t = (np.asarray(r, dtype=np.float64) - self.r0) / (0.5 - self.r0)
        return np.polynomial.polynomial.polyval(t, self.coef)

    def __call__(self, r):
        r = np.asarray(r, dtype=np.float64)
        out = self.K(r)
        if self.coef_I is not None:
            out = np.where(r <= self.eps_I, self.T_I(np.minimum(r, self.eps_I)), out)
        if self.coef is None:
            # eps_B = 0: no transition region; constant K(1/2) beyond radius 1/2
            return np.where(r <= 0.5, out, self.k_half)
        mid = (r > self.r0) & (r <= 0.5)
        out = np.where(mid, self.T_B(r), out)
        out = np.where(r > 0.5, self.T_B(0.5), out)
        return out


# ---- eq. b_l::K_RF: Fourier coefficients by the trapezoidal rule ------------

def index_set(N: int):
    """I_N in one dimension: -N/2, ..., N/2 - 1."""
    return np.arange(-N // 2, N // 2)


def coefficients(sigma: float, N: int, d: int, eps_B: float, p: int,
                 kind: str = "gaussian", eps_I: float = 0.0) -> np.ndarray:
    """b_l for l in I_N^d, array of shape (N,)*d indexed by l + N/2.

    b_l = N^{-d} sum_{j in I_N^d} K_R(j/N) exp(-2 pi i j.l/N), computed as a DFT
    (numpy's FFT as the library primitive) of the samples placed at j mod N."""
    K = RegKernel(sigma, eps_B, p, kind, eps_I)
    j = index_set(N)
    grids = np.meshgrid(*([j / N] * d), indexing="ij")
    r = np.sqrt(sum(g * g for g in grids))
    S = K(r)                              # indexed by j + N/2
    S_mod = np.fft.ifftshift(S)           # indexed by j mod N
    F = np.fft.fftn(S_mod) / float(N) ** d
    b = np.fft.fftshift(F)                # indexed by l + N/2
    if np.abs(b.imag).max() > 1e-12 * max(1.0, np.abs(b.real).max()):
        raise AssertionError("b_l not real: samples are not even")
    return np.ascontiguousarray(b.real)


def K_RF(y, bhat: np.ndarray, N: int):
    """sum_{l in I_N^d} b_l exp(2 pi i l.y) at points y (m x d), complex
    (eq. K_RF), evaluated separably: exp(2 pi i l.y) = prod_t exp(2 pi i l_t y_t)."""
    y = np.asarray(y, dtype=np.float64)
    if y.ndim == 1:
        y = y[:, None]
    E = _phases(y, N, +1.0)
    B = bhat.reshape(N, -1).astype(np.complex128)
    out = np.empty(y.shape[0], dtype=np.complex128)
    for s in range(0, y.shape[0], 1024):
        rows = np.arange(s, min(y.shape[0], s + 1024))
        P = _outer_rest(E, rows)
        out[rows] = (E[0][rows] * (P @ B.T)).sum(axis=1)
    return out


# ---- the exact trigonometric operator of Alg. nfft_fastsum -----------------

def _phases(vt, N, sign):
    l = index_set(N)
    return [np.exp(sign * 2j * np.pi * np.outer(vt[:, t], l)) for t in range(vt.shape[1])]


def _outer_rest(E, rows):
    """Row-wise outer product of E[1:], flattened: (len(rows), N^(d-1))."""
    if len(E) == 1:
        return np.ones((len(rows), 1), dtype=np.complex128)
    P = E[1][rows]
    for t in range(2, len(E)):
        P = (P[:, :, None] * E[t][rows][:, None, :]).reshape(len(rows), -1)
    return P


def trig_operator(vt, x, bhat: np.ndarray, N: int, chunk: int = 1024, targets=None):
    """f_j = Re sum_{l in I_N^d} b_l xhat_l exp(2 pi i l.t_j), with the adjoint
    sum xhat_l = sum_i x_i exp(-2 pi i l.v_i) (steps 1-3 of Alg. nfft_fastsum
    with both nonequispaced sums done exactly).  With the targets t_j equal to
    the sources (default) this approximates W~ x; otherwise
    sum_i x_i K(t_j - v_i).

    vt: scaled source nodes (n x d); x: (n,) or (nvec, n); targets: scaled
    target nodes (n_t x d) or None."""
    vt = np.asarray(vt, dtype=np.float64)
    if vt.ndim == 1:
        vt = vt[:, None]
    n, d = vt.shape
    tt = vt if targets is None else np.asarray(targets, dtype=np.float64).reshape(-1, d)
    nt = tt.shape[0]
    X = np.asarray(x, dtype=np.float64)
    single = X.ndim == 1
    X = X.reshape(1, n) if single else X
    Em = _phases(vt, N, -1.0)
    Ep = _phases(tt, N, +1.0)
    outs = []
    B = bhat.reshape(N, -1)
    for xv in X:
        xhat = np.zeros((N, N ** (d - 1)), dtype=np.complex128)
        for s in range(0, n, chunk):
            rows = np.arange(s, min(n, s + chunk))
            P = _outer_rest(Em, rows)
            xhat += (xv[rows, None] * Em[0][rows]).T @ P
        F = B * xhat
        f = np.empty(nt)
        for s in range(0, nt, chunk):
            rows = np.arange(s, min(nt, s + chunk))
            P = _outer_rest(Ep, rows)
            Q = P @ F.T                                   # (rows, N)
            f[rows] = (Ep[0][rows] * Q).sum(axis=1).real
        outs.append(f)
    return outs[0] if single else np.stack(outs)


def trig_matrix(vt, bhat: np.ndarray, N: int):
    """The n x n matrix of the exact trigonometric operator (small n):
    M_ji = Re K_RF(v_j - v_i)."""
    vt = np.asarray(vt, dtype=np.float64)
    if vt.ndim == 1:
        vt = vt[:, None]
    n, d = vt.shape
    Ep = _phases(vt, N, +1.0)
    Eall = _outer_rest(Ep, np.arange(n))
    Efull = (Ep[0][:, :, None] * Eall[:, None, :]).reshape(n, -1)  # exp(2 pi i l.v_j)
    b = bhat.reshape(-1)
    return ((Efull * b[None, :]) @ Efull.conj().T).real


# ---- Alg. nfft_normalized_matvec with the exact trigonometric operator -----

class TrigGraph:
    """Steps 1-5 of Alg. nfft_normalized_matvec with Alg. nfft_fastsum replaced
    by its exact trigonometric operator.  apply_Wt approximates W~ = W + K(0) I
    in the original coordinates (for the Gaussian K(0) = 1)."""

    def __init__(self, v, sigma: float, N: int, eps_B: float, p: int, kind: str = "gaussian",
                 eps_I: float = 0.0):
        self.c, self.rho, self.vt = scaling(v, eps_B)
        self.kind = kind
        self.sigma_t = scaled_param(kind, sigma, self.rho)
        self.scale = output_scale(kind, self.rho)
        self.K0 = float(radial_kernel(kind, sigma)(0.0))
        self.N = N
        self.reg = RegKernel(self.sigma_t, eps_B, p, kind, eps_I)
        self.bhat = coefficients(self.sigma_t, N, self.vt.shape[1], eps_B, p, kind, eps_I)
        ones = np.ones(self.vt.shape[0])
        self.d = self.apply_Wt(ones) - self.K0                       # step 4
        self.dinv = 1.0 / np.sqrt(self.d)

    def apply_Wt(self, x):
        f = trig_operator(self.vt, x, self.bhat, self.N)
        if self.reg.coef_I is not None:
            f = f + self.near_field(x)
        return self.scale * f

    def near_field(self, x):
        """sum over pairs with ||v~_j - v~_i|| <= eps_I (i = j included) of
        x_i (K - K_R)(v~_j - v~_i): the correction that restores K near 0."""
        X = np.asarray(x, dtype=np.float64)
        out = np.zeros(self.vt.shape[0])
        for s in range(0, self.vt.shape[0], 512):
            r = np.sqrt(((self.vt[s:s + 512, None, :] - self.vt[None, :, :]) ** 2).sum(axis=2))
            out[s:s + 512] = self.reg.near(r) @ X
        return out

    def apply_W(self, x):
        return self.apply_Wt(x) - self.K0 * np.asarray(x, dtype=np.float64)

    def apply_A(self, x):                                             # step 5
        xs = self.dinv * np.asarray(x, dtype=np.float64)
        return self.dinv * (self.apply_Wt(xs) - self.K0 * xs)

    def apply_Ls(self, x):
        return np.asarray(x, dtype=np.float64) - self.apply_A(x)


# ---- Section 3.1: error quantities ------------------------------------------

def kerr_sampled(bhat, N, sigma, eps_B, d, samples=20000, seed=0, kind="gaussian"):
    """max |K(y) - Re K_RF(y)| over random y with ||y|| <= 1/2 - eps_B
    (eq. KERR_estimate, maximum discretised by sampling); K of the given kind
    with parameter sigma (in the scaled coordinates)."""
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(samples, d))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = (0.5 - eps_B) * rng.uniform(0.0, 1.0, size=samples) ** (1.0 / d)
    y = g * r[:, None]
    return float(np.abs(radial_kernel(kind, sigma)(r) - K_RF(y, bhat, N).real).max())


def lemma_bound(eps: float, eta: float) -> float:
    """Lemma normalization_propagation: ||A - A_E||_inf <= eps (1 + eta) / (eta (eta - eps))."""
    if not eps < eta:
        return math.inf
    return eps * (1.0 + eta) / (eta * (eta - eps))
