"""Python handle on the FP64 CPU oracle (``libmbh_oracle.so``).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It marshals numpy
arrays into the C oracle, which implements the likelihood of arXiv:2005.01827
Sec. II step by step (see the header of ``mbh_oracle.c``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mbh_oracle.c")
CFLAGS = ["-O3", "-march=native", "-ffp-contract=off", "-std=gnu11", "-Wall", "-fopenmp", "-fPIC", "-shared"]


def _host_tag() -> str:
    """Short tag of this host's CPU model and instruction-set flags: the
    library is built with -march=native, so each kind of host builds its
    own copy instead of loading one built for another CPU."""
    import hashlib
    model, flags = "", ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not model and line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                elif not flags and line.startswith("flags"):
                    flags = line.split(":", 1)[1].strip()
                if model and flags:
                    break
    except OSError:
        pass
    return hashlib.sha1((model + "|" + flags).encode()).hexdigest()[:12]


_LIB_PATH = os.path.join(_HERE, f"libmbh_oracle_{_host_tag()}.so")

SUPPORTED_MODES = ((2, 2), (3, 3), (4, 4), (2, 1), (3, 2), (4, 3))

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: -O3 -march=native, FMA contraction off
    (plain IEEE double operations, no fast-math), OpenMP over walkers."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_source.argtypes = [_dp, ctypes.c_double, _dp]
        L.oracle_mode.argtypes = [_dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  _dp, _dp, _dp, _dp, _dp]
        L.oracle_phase22_pieces.argtypes = [_dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.oracle_amp22.argtypes = [_dp, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
        L.oracle_swsh.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_lisa_positions.argtypes = [ctypes.c_double, _dp]
        L.oracle_link.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        L.oracle_response.argtypes = [_dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, _dp]
        L.oracle_tdi.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp, _dp, _dp]
        L.oracle_mode_weights.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_tridiag.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        L.oracle_spline_coeffs.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.oracle_spline_eval.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp]
        L.oracle_sparse.argtypes = [_dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, _ip,
                                    ctypes.c_int, ctypes.c_double, _lp, _dp, _dp, _dp, _dp]
        L.oracle_template.argtypes = [_dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                      _ip, ctypes.c_int, ctypes.c_double, _dp]
        L.oracle_loglike.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                     _dp, _dp, ctypes.c_int, _ip, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _modes(modes):
    m = np.ascontiguousarray(np.asarray(modes, dtype=np.int32).reshape(-1, 2))
    return m, m.ctypes.data_as(_ip), m.shape[0]


def _check(st, what):
    if st != 0:
        raise ValueError(f"oracle {what} rejected its arguments (status {st})")


SOURCE_FIELDS = ("M", "eta", "delta", "Dl", "tcoal", "af", "Mfin", "fRD", "fd", "fJ", "fpeak",
                 "A0", "cR", "b1", "b0", "kRD")


def source(theta, t0):
    th = _f64(theta)
    out = np.zeros(16)
    _check(lib().oracle_source(_d(th), t0, _d(out)), "source")
    return dict(zip(SOURCE_FIELDS, out))


def mode(theta, t0, l, m, f):
    th, f = _f64(theta), _f64(f)
    A, phi, dphi, t = (np.zeros(f.size) for _ in range(4))
    _check(lib().oracle_mode(_d(th), t0, l, m, f.size, _d(f), _d(A), _d(phi), _d(dphi), _d(t)), "mode")
    return A, phi, dphi, t


def phase22_pieces(theta, t0, which, f):
    th, f = _f64(theta), _f64(f)
    out = np.zeros((f.size, 3))
    _check(lib().oracle_phase22_pieces(_d(th), t0, which, f.size, _d(f), _d(out)), "phase22_pieces")
    return out


def amp22(theta, t0, f):
    th, f = _f64(theta), _f64(f)
    A, g = np.zeros(f.size), np.zeros(f.size)
    _check(lib().oracle_amp22(_d(th), t0, f.size, _d(f), _d(A), _d(g)), "amp22")
    return A, g


def swsh(l, m, theta, phi):
    out = np.zeros(2)
    _check(lib().oracle_swsh(l, m, theta, phi, _d(out)), "swsh")
    return complex(out[0], out[1])


def lisa_positions(t):
    out = np.zeros(9)
    _check(lib().oracle_lisa_positions(t, _d(out)), "lisa_positions")
    return out.reshape(3, 3)


def link(f, t, lam, beta, psi, r, s, cross):
    out = np.zeros(2)
    _check(lib().oracle_link(f, t, lam, beta, psi, r, s, cross, _d(out)), "link")
    return complex(out[0], out[1])


def response(theta, t0, l, m, f, t):
    th = _f64(theta)
    out = np.zeros(7)
    _check(lib().oracle_response(_d(th), t0, l, m, f, t, _d(out)), "response")
    return out[0:6:2] + 1j * out[1:6:2], out[6]


def tdi(f, t, lam, beta, psi, kp, kc):
    """A, E, T transfer for explicit plus/cross weights; returns (aet[3], orbital phase)."""
    kp_ = np.array([complex(kp).real, complex(kp).imag])
    kc_ = np.array([complex(kc).real, complex(kc).imag])
    out = np.zeros(7)
    _check(lib().oracle_tdi(f, t, lam, beta, psi, _d(kp_), _d(kc_), _d(out)), "tdi")
    return out[0:6:2] + 1j * out[1:6:2], out[6]


def mode_weights(l, m, iota, phiref):
    out = np.zeros(4)
    _check(lib().oracle_mode_weights(l, m, iota, phiref, _d(out)), "mode_weights")
    return complex(out[0], out[1]), complex(out[2], out[3])


def tridiag(sub, dia, sup, rhs):
    sub, dia, sup, rhs = map(_f64, (sub, dia, sup, rhs))
    x = np.zeros(rhs.size)
    _check(lib().oracle_tridiag(rhs.size, _d(sub), _d(dia), _d(sup), _d(rhs), _d(x)), "tridiag")
    return x


def spline_coeffs(x, y):
    x, y = _f64(x), _f64(y)
    c = np.zeros((x.size - 1, 4))
    _check(lib().oracle_spline_coeffs(x.size, _d(x), _d(y), _d(c)), "spline_coeffs")
    return c


def spline_eval(x, coef, xq):
    x, coef, xq = _f64(x), _f64(coef), _f64(xq)
    yq = np.zeros(xq.size)
    _check(lib().oracle_spline_eval(x.size, _d(x), _d(coef), xq.size, _d(xq), _d(yq)), "spline_eval")
    return yq


def sparse(theta, grid, modes=SUPPORTED_MODES, ns=256, t0=0.0):
    """Sparse stage of one walker: bands, knots, functions, spline coefficients."""
    th = _f64(theta)
    m, mp, nm = _modes(modes)
    band = np.zeros((nm, 4), dtype=np.int64)
    fband = np.zeros((nm, 2))
    f = np.zeros((nm, ns))
    fn = np.zeros((nm, 8, ns))
    cf = np.zeros((nm, 8, ns - 1, 4))
    _check(lib().oracle_sparse(_d(th), grid.df, grid.k0, grid.n, nm, mp, ns, t0,
                               band.ctypes.data_as(_lp), _d(fband), _d(f), _d(fn), _d(cf)), "sparse")
    return dict(band=band, fband=fband, f=f, fn=fn, cf=cf)


def template(theta, grid, modes=SUPPORTED_MODES, ns=256, t0=0.0):
    """Dense template h[3][n] (complex128) of one walker."""
    th = _f64(theta)
    m, mp, nm = _modes(modes)
    h = np.zeros((3, grid.n, 2))
    _check(lib().oracle_template(_d(th), grid.df, grid.k0, grid.n, nm, mp, ns, t0, _d(h)), "template")
    return h[..., 0] + 1j * h[..., 1]


def loglike(theta, grid, data, psd, modes=SUPPORTED_MODES, ns=256, t0=0.0, nthreads=0):
    """ln L and the per-channel <d|h>, <h|h> for a batch theta[B][11].

    Returns out[B][7] = (lnL, DH_A, DH_E, DH_T, HH_A, HH_E, HH_T)."""
    th = _f64(np.atleast_2d(theta))
    B = th.shape[0]
    d = np.ascontiguousarray(np.stack([np.asarray(data).real, np.asarray(data).imag], axis=-1), dtype=np.float64)
    S = _f64(psd)
    assert d.shape == (3, grid.n, 2) and S.shape == (3, grid.n)
    m, mp, nm = _modes(modes)
    out = np.zeros((B, 7))
    _check(lib().oracle_loglike(B, _d(th), grid.df, grid.k0, grid.n, _d(d), _d(S), nm, mp, ns, t0,
                                nthreads, _d(out)), "loglike")
    return out
