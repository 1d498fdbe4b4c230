"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, rejects bad arguments without touching a GPU, and its host
FP64 filter matches the oracle's coefficients divided by the window
transform (computed here by quadrature of the Kaiser-Bessel window)."""
import math
import os
import re

import numpy as np
import pytest

import paper_1808_04580_amd as nfl
from oracle import fastsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "nfl.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nfl_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = nfl.lib()
    syms = header_symbols()
    assert len(syms) >= 19
    for s in syms:
        assert hasattr(L, s), s
        assert s in nfl.SIGNATURES, "binding lacks " + s


def test_error_codes_without_gpu():
    L = nfl.lib()
    import ctypes
    h = ctypes.c_void_p()
    assert L.nfl_create(ctypes.byref(h), 4, None) == nfl.NFL_ERR_ARG
    assert L.nfl_create(None, 3, None) == nfl.NFL_ERR_ARG
    assert L.nfl_set_points(None, 10, None) == nfl.NFL_ERR_ARG
    assert L.nfl_apply_Ls(None, None, None, 1, 10) == nfl.NFL_ERR_ARG
    for c in [0, 1, -1, -2, -3, -4, -5, -6]:
        assert nfl.strerror(c) and "unknown" not in nfl.strerror(c)
    out = np.empty(10)
    assert L.nfl_compute_filter(3, 15, 4, 4, 0.0, 0.1, out.ctypes.data_as(ctypes.c_void_p), 10) \
        == nfl.NFL_ERR_ARG
    # batches, the accuracy probe and the tuner reject null handles / bad
    # arguments before touching a device
    b = ctypes.c_void_p()
    assert L.nfl_batch_create(None, None, 1, 1, None) == nfl.NFL_ERR_ARG
    assert L.nfl_batch_create(ctypes.byref(b), None, 0, 8, None) == nfl.NFL_ERR_ARG
    assert L.nfl_batch_apply_Ls(None, None, None) == nfl.NFL_ERR_ARG
    assert L.nfl_batch_offsets(None, None, 0) == nfl.NFL_ERR_ARG
    assert L.nfl_batch_info(None, None, None, None, None) == nfl.NFL_ERR_ARG
    assert L.nfl_batch_destroy(None) == nfl.NFL_OK
    assert L.nfl_direct_rows(None, 0.1, None, None, 1, None, None) == nfl.NFL_ERR_ARG
    assert L.nfl_autotune(None, 0.1, 1e-5, 64, 1, None, None, None, None, None, None, None,
                          None) == nfl.NFL_ERR_ARG
    assert L.nfl_set_option(None, nfl.OPT_KERNEL, 2) == nfl.NFL_ERR_ARG
    assert L.nfl_nystrom(None, None, 0, 1, 1, 1, None, None, None) == nfl.NFL_ERR_ARG
    assert L.nfl_set_kernel_ex(None, 1, 0.1, 32, 4, 0.0) == nfl.NFL_ERR_ARG
    assert L.nfl_krr_solve(None, 1.0, None, None, 0, 1e-6, 10, None, None) == nfl.NFL_ERR_ARG
    assert L.nfl_set_points_frame(None, 1, None, None) == nfl.NFL_ERR_ARG
    assert L.nfl_evaluate(None, None, None, None) == nfl.NFL_ERR_ARG


def kb_hat_quadrature(xi, m, b=1.5 * math.pi, nq=2001):
    """Fourier transform of psi(t) = sinh(b sqrt(m^2-t^2))/(sqrt(m^2-t^2) b e^{bm})
    on [-m, m] by the composite Simpson rule after t = m sin(theta), which turns
    the integrand into the smooth sinh(b m cos theta) cos(2 pi xi m sin theta)."""
    th = np.linspace(-math.pi / 2, math.pi / 2, nq)
    f = np.sinh(b * m * np.cos(th)) * np.cos(2 * math.pi * xi * m * np.sin(th))
    h = th[1] - th[0]
    return h / 3 * (f[0] + f[-1] + 4 * f[1:-1:2].sum() + 2 * f[2:-1:2].sum()) / (b * math.exp(b * m))


def kb_psi(t, m, b=1.5 * math.pi):
    t = np.asarray(t, dtype=np.float64)
    s = np.sqrt(np.maximum(m * m - t * t, 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(s > 0, np.sinh(b * s) / np.where(s > 0, s, 1.0), b) / (b * math.exp(b * m))


def poly_window(coef, m, t):
    """The piecewise polynomial window at grid offsets t in (-m, m]."""
    t = np.asarray(t, dtype=np.float64)
    c = np.ceil(t + m).astype(int) - 1          # t in (c - m, c - m + 1]
    f = (c - (m - 1)) - t                       # fraction in [0, 1)
    g = 2 * f - 1
    out = np.zeros_like(t)
    for q in range(coef.shape[1] - 1, -1, -1):
        out = out * g + coef[c, q].astype(np.float64)
    return out


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7, 8])
def test_window_polynomials_match_kaiser_bessel(m):
    """The polynomial window (degree 7 per unit interval) equals the
    Kaiser-Bessel window to float32 level: within 1e-7 of psi(0) for m >= 3,
    4e-7 for m = 2 (whose own NFFT error, ~1e-3, is far larger)."""
    coef = nfl.window_coefficients(m)
    assert coef.shape == (2 * m, nfl.WIN_NC)
    t = np.linspace(-m + 1e-9, m, 20001)
    err = np.abs(poly_window(coef, m, t) - kb_psi(t, m)).max() / kb_psi(0.0, m)
    assert err < (4e-7 if m == 2 else 1e-7), err


def poly_window_hat(coef, m, xi, nq=64):
    """Transform of the piecewise polynomial window, Gauss-Legendre per interval."""
    x, w = np.polynomial.legendre.leggauss(nq)
    acc = 0.0
    for c in range(2 * m):
        t = (c - m) + 0.5 * (x + 1.0)             # (c - m, c - m + 1)
        acc += 0.5 * np.sum(w * poly_window(coef, m, t) * np.cos(2 * math.pi * xi * t))
    return acc


@pytest.mark.parametrize("d,N,m,eps", [(1, 16, 3, 0.0), (2, 16, 4, 0.125), (3, 8, 2, 0.25)])
def test_filter_equals_coefficients_over_window_transform(d, N, m, eps):
    sig = 0.12
    p = m
    F = nfl.compute_filter(d, N, m, p, eps, sig)
    b = fastsum.coefficients(sig, N, d, eps, p)           # indexed by l + N/2 on I_N^d
    nos = 2 * N
    coef = nfl.window_coefficients(m)
    wh = np.array([poly_window_hat(coef, m, l / nos) for l in range(-N // 2, N // 2 + 1)])
    # the transform of the polynomial window is the Kaiser-Bessel one to float32 level
    wkb = np.array([kb_hat_quadrature(l / nos, m) for l in range(-N // 2, N // 2 + 1)])
    assert np.abs(wh / wkb - 1).max() < 1e-6
    # expected on the extended set {-N/2..N/2}^(d-1) x {0..N/2}: real part of
    # the asymmetric sum = b_l split evenly between l and -l at the Nyquist indices
    ext = np.arange(-N // 2, N // 2 + 1)
    grids = np.meshgrid(*([ext] * (d - 1) + [np.arange(0, N // 2 + 1)]), indexing="ij")
    L = np.stack(grids, axis=-1).reshape(-1, d)
    exp = np.empty(L.shape[0])
    for q, l in enumerate(L):
        inI = np.all(l <= N // 2 - 1)
        inmI = np.all(-l <= N // 2 - 1)
        val = 0.0
        if inI:
            val += 0.5 * b[tuple(l + N // 2)]
        if inmI:
            val += 0.5 * b[tuple(-l + N // 2)]
        den = np.prod([wh[li + N // 2] ** 2 for li in l])
        exp[q] = val / den
    np.testing.assert_allclose(F.reshape(-1), exp, rtol=1e-10, atol=1e-12 * np.abs(exp).max())


@pytest.mark.parametrize("kind,d,N,m,eps", [("multiquadric", 2, 16, 4, 0.125),
                                            ("inverse_multiquadric", 3, 8, 3, 0.25),
                                            ("laplacian_rbf", 2, 16, 4, 0.125)])
def test_filter_other_kernels_equals_coefficients_over_window_transform(kind, d, N, m, eps):
    """The library's host filter for the other kernels (derivatives by a
    power-series recurrence) against the oracle's coefficients (derivatives
    by the binomial series), divided by K(0) and the squared window
    transform, at the interior frequencies."""
    c = 0.12
    p = m
    eps_I = p / N if kind == "laplacian_rbf" else 0.0    # inner regularisation (Laplacian RBF)
    F = nfl.compute_filter(d, N, m, p, eps, c, kind=kind, eps_I=eps_I)
    K0 = float(fastsum.radial_kernel(kind, c)(0.0))
    b = fastsum.coefficients(c, N, d, eps, p, kind, eps_I) / K0
    nos = 2 * N
    coef = nfl.window_coefficients(m)
    wh = np.array([poly_window_hat(coef, m, l / nos) for l in range(-N // 2, N // 2 + 1)])
    ext = np.arange(-N // 2, N // 2 + 1)
    grids = np.meshgrid(*([ext] * (d - 1) + [np.arange(0, N // 2 + 1)]), indexing="ij")
    L = np.stack(grids, axis=-1).reshape(-1, d)
    exp = np.empty(L.shape[0])
    for q, l in enumerate(L):
        val = 0.0
        if np.all(l <= N // 2 - 1):
            val += 0.5 * b[tuple(l + N // 2)]
        if np.all(-l <= N // 2 - 1):
            val += 0.5 * b[tuple(-l + N // 2)]
        exp[q] = val / np.prod([wh[li + N // 2] ** 2 for li in l])
    np.testing.assert_allclose(F.reshape(-1), exp, rtol=1e-9, atol=1e-11 * np.abs(exp).max())
