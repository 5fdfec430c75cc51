"""Oracle: plain, slow, obviously-correct CPU references for everything the
product computes.  TEST INFRASTRUCTURE ONLY -- the product package never
imports this module; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

Contents (each cites the passage it follows):

* ``xcorr2d`` / ``conv_nhwc``      -- FP64 convolution (C library, ``xcorr_oracle.c``)
* ``conv_nhwc_at``                -- the multi-channel definition at selected output pixels
* ``xcorr2d_loops``               -- the same definition as pure-Python loops (tiny inputs)
* ``power_model``                 -- Eq. 2 / Eq. 3 model, energy estimate, optimal clock,
                                     clock band, least-squares fit (section III.A and the
                                     "Model-steered frequency tuning" subsection)
* ``measure``                     -- energy from a power trace (section III.A), metrics and
                                     objective selection (section III.C)
* ``space``                       -- the restricted Cartesian tune space (section IV)

The oracle shares no code with the HIP path: no header, helper, table or
constant generator.  It is pinned by ``tests/test_oracle_*.py`` against brute
force, closed forms and invariants.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xcorr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile the C oracle with gcc (-O2, OpenMP).  Called by the repo's
    build step; also on first use if the library is missing."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, fp, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
        lib.oracle_xcorr2d_f64.argtypes = [fp, i64, i64, fp, i64, i64, dp, ctypes.c_int]
        lib.oracle_xcorr2d_f64.restype = ctypes.c_int
        lib.oracle_conv_nhwc_f64.argtypes = [fp, i64, i64, i64, i64, fp, i64, i64, i64, i64, i64,
                                             dp, ctypes.c_int]
        lib.oracle_conv_nhwc_f64.restype = ctypes.c_int
        lib.oracle_conv_nhwc_points_f64.argtypes = [fp, i64, i64, i64, i64, fp, i64, i64, i64, i64, i64,
                                                    ctypes.POINTER(ctypes.c_int64), i64, dp, ctypes.c_int]
        lib.oracle_conv_nhwc_points_f64.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def max_threads():
    return _load().oracle_max_threads()


def xcorr2d(image, weights, nthreads=0):
    """Single-channel 2-D cross-correlation, valid region, no filter flip,
    accumulated in FP64 over the exact FP64 widening of the FP32 inputs.
    ``image`` is (oh+fh-1, ow+fw-1); returns (oh, ow) float64."""
    img, pi = _f32(image)
    w, pw = _f32(weights)
    (ih, iw), (fh, fw) = img.shape, w.shape
    out = np.empty((ih - fh + 1, iw - fw + 1), dtype=np.float64)
    rc = _load().oracle_xcorr2d_f64(pi, ih, iw, pw, fh, fw,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nthreads)
    if rc != 0:
        raise ValueError("bad xcorr2d sizes")
    return out


def conv_nhwc(x, wt, pad_h, pad_w, nthreads=0):
    """Multi-channel convolution (cross-correlation), stride 1, zero padding.
    x: [n][h][w][c_in]; wt: [c_out][fh][fw][c_in]; returns [n][oh][ow][c_out]
    float64.  BF16 inputs are passed as their exact FP32 values."""
    xa, px = _f32(x)
    wa, pk = _f32(wt)
    n, h, w, ci = xa.shape
    co, fh, fw, ci2 = wa.shape
    if ci != ci2:
        raise ValueError("channel mismatch")
    oh, ow = h + 2 * pad_h - fh + 1, w + 2 * pad_w - fw + 1
    out = np.empty((n, oh, ow, co), dtype=np.float64)
    rc = _load().oracle_conv_nhwc_f64(px, n, h, w, ci, pk, co, fh, fw, pad_h, pad_w,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nthreads)
    if rc != 0:
        raise ValueError("bad conv sizes")
    return out


def conv_nhwc_at(x, wt, pad_h, pad_w, points, nthreads=0):
    """conv_nhwc at selected output pixels: points is a sequence of (b, y, x);
    returns [len(points)][c_out] float64."""
    xa, px = _f32(x)
    wa, pk = _f32(wt)
    n, h, w, ci = xa.shape
    co, fh, fw, ci2 = wa.shape
    if ci != ci2:
        raise ValueError("channel mismatch")
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.int64).reshape(-1, 3))
    out = np.empty((pts.shape[0], co), dtype=np.float64)
    rc = _load().oracle_conv_nhwc_points_f64(px, n, h, w, ci, pk, co, fh, fw, pad_h, pad_w,
                                             pts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), pts.shape[0],
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nthreads)
    if rc != 0:
        raise ValueError("bad conv sizes or points")
    return out


def xcorr2d_loops(image, weights):
    """The definition as pure-Python loops, for tiny inputs only."""
    ih, iw = len(image), len(image[0])
    fh, fw = len(weights), len(weights[0])
    out = []
    for y in range(ih - fh + 1):
        row = []
        for x in range(iw - fw + 1):
            s = 0.0
            for i in range(fh):
                for j in range(fw):
                    s += float(image[y + i][x + j]) * float(weights[i][j])
            row.append(s)
        out.append(row)
    return out


def max_rel_err(got, ref):
    """Normwise relative error max|g-r| / max|r| (the parity metric)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref)) if ref.size else 0.0
    if ref.size == 0:
        return 0.0
    num = np.max(np.abs(got - ref))
    return float(num / den) if den > 0 else float(num)
