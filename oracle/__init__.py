"""The oracle: a plain, slow, obviously correct FP64 CPU implementation of
what the HIP library computes.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import, call, link or execute anything in this package.  The
library's product path never routes through it, and the two share no code:
no kernels, headers, helpers, tables or constant generators.  The only input
both sides see is the seeded synthetic data from ``synth``.

Modules
-------
``graph``    the weighted graph of Section 2 by direct O(n^2) sums in FP64
             (weights eq. W_gaussian, degree, L = D - W, L_s of eq. nomlap,
             A = D^{-1/2} W D^{-1/2}); the O(n^2) loops live in ``direct.c``.
``fastsum``  the trigonometric kernel approximation of Section 3: node
             scaling (Alg. nfft_normalized_matvec steps 1-2), the regularised
             kernel K_R, its Fourier coefficients (eq. b_l::K_RF) and the exact
             trigonometric operator that Alg. nfft_fastsum approximates,
             evaluated by direct nonequispaced DFTs; plus the a-posteriori
             error quantities of Section 3.1.
``krylov``   Lanczos with full reorthogonalisation (Section 4) and CG for the
             kernel-SSL system (eq. ssl::system).
``mlp``      FP64 reference of the pointwise warm-start network.
``krr``      kernel ridge regression (Section 6.3): (K + beta I) alpha = f by
             a dense solve, and the prediction sum.
``nystrom``  the Nystrom-Gaussian-NFFT eigenvalue approximation (Alg.
             nystrom_hybrid, Section 5.2), steps 3-8 on a given operator.

Parity pins
-----------
Every function is pinned in ``tests/test_oracle_pins.py`` against something
other than itself: closed forms, brute force on tiny inputs, identities of
Section 2, special cases that reduce to numpy/LAPACK routines, and the Lemma
of Section 3.1.  Functions without such a pin say "parity unpinned" here:
(none at present).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "_direct.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile direct.c with gcc (FP64, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64, dbl, ip = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.oracle_w_rows.argtypes = [i64, ctypes.c_int, ip, dbl, ctypes.c_int, ip, i64, ip, ip]
        L.oracle_w_rows.restype = ctypes.c_int
        L.oracle_degree_rows.argtypes = [i64, ctypes.c_int, ip, dbl, i64, ip, ip]
        L.oracle_degree_rows.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().oracle_num_threads())
