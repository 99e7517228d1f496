"""FP64 CPU oracle for the adaptive-force-update gravity path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the HIP path.  Each wrapper below calls the plain C
routine of the same name in ``oracle.c`` (built into ``liboracle.so`` by
:func:`build`), which states the definition it implements:

* :func:`field` / :func:`direct` -- softened direct sum for the acceleration,
  the jerk (the particle discretisation of the jerk integral, Eq. 5) and the
  tidal tensor (whose Frobenius norm enters Eq. 7); optionally in a periodic
  cube with every pair at its nearest image (how the paper treats the jerk
  of periodic problems, Sec. 3.4); :func:`direct_soft` with a softening length
  per particle (each pair takes the mean of its two kernels), and
  :func:`neighbour_length`, the k-th neighbour distance those lengths
  follow (plain numpy).
* :func:`timestep` -- the tidal timestep of Eq. 7 and its power-of-two bin.
* :func:`select` -- force-age counter (Eq. 3) and update condition (Eq. 4).
* :func:`predict` -- jerk predictor (Eq. 6) in closed form ``a0 + j (t - t0)``.
* :func:`force_log` / :func:`predict_poly` -- the alternative to Eq. 6 that
  Sec. 2.2 names: extrapolate g from a few logged past values with an
  interpolating polynomial (plain numpy, written here rather than in C).
* :func:`adjoint` -- exact gradient of ``L = sum_i w_i . a_i``.
* :func:`moments` -- node multipoles (mass, centre of mass, mean velocity,
  traceless quadrupole and its rate) of a particle set.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# Compiled for the generic x86-64-v3 level (any recent EPYC/Xeon host) with
# fused multiply-add contraction off, so every operation is rounded once as
# written in the C source.
CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.orc_kernel.argtypes = [I64, P, D, P, P, P]
        lib.orc_field.argtypes = [I64, P, P, P, D, D, I64, P, P, P, P, P, P]
        lib.orc_direct.argtypes = [I64, P, P, P, D, D, I64, P, P, P, P]
        lib.orc_abs_scale.argtypes = [I64, P, P, D, D, I64, P, P]
        lib.orc_field_box.argtypes = [I64, P, P, P, D, D, D, I64, P, P, P, P, P, P]
        lib.orc_direct_box.argtypes = [I64, P, P, P, D, D, D, I64, P, P, P, P]
        lib.orc_abs_scale_box.argtypes = [I64, P, P, D, D, D, I64, P, P]
        lib.orc_field_soft.argtypes = [I64, P, P, P, P, D, I64, P, P, P, P, P, P, P]
        lib.orc_ewald_unit.argtypes = [I64, P, D, D, ctypes.c_int, ctypes.c_int, P, P, P, P]
        lib.orc_direct_ewald.argtypes = [I64, P, P, P, D, D, D, I64, P, P, P, P]
        lib.orc_timestep.argtypes = [I64, P, D, D, ctypes.c_int32, P, P]
        lib.orc_select.argtypes = [I64, P, P, I64, ctypes.c_int32, D, P]
        lib.orc_select.restype = I64
        lib.orc_predict.argtypes = [I64, P, P, P, D, P]
        lib.orc_adjoint.argtypes = [I64, P, P, P, D, D, I64, P, P, P]
        lib.orc_moments.argtypes = [I64, P, P, P, P, P]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(k: int) -> None:
    """Use ``k`` OpenMP threads in later calls (``k <= 0``: the default)."""
    _load().orc_set_threads(int(k))


def kernel(r, h):
    """Return (f, D, W) of the cubic-spline kernel at separations ``r``."""
    r = _f64(r).ravel()
    f = np.empty_like(r)
    D = np.empty_like(r)
    W = np.empty_like(r)
    _load().orc_kernel(r.size, _ptr(r), float(h), _ptr(f), _ptr(D), _ptr(W))
    return f, D, W


def field(x, v, m, eps, G, p, pv=None, excl=None, box=0.0):
    """Acceleration, jerk and tidal tensor at probe points ``p`` (np x 3).
    box > 0: every pair at its nearest periodic image in a cube of that side."""
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    m = _f64(m).ravel()
    p = _f64(p, (-1, 3))
    pv = np.zeros_like(p) if pv is None else _f64(pv, (-1, 3))
    ex = None if excl is None else np.ascontiguousarray(excl, dtype=np.int64)
    k = p.shape[0]
    acc = np.empty((k, 3))
    jerk = np.empty((k, 3))
    tid = np.empty((k, 6))
    _load().orc_field_box(x.shape[0], _ptr(x), _ptr(v), _ptr(m), float(eps), float(G), float(box),
                          k, _ptr(p), _ptr(pv), _ptr(ex), _ptr(acc), _ptr(jerk), _ptr(tid))
    return acc, jerk, tid


def direct(x, v, m, eps, G, targets=None, box=0.0, ewald=False):
    """Direct sum at particles ``targets`` (default: all), self excluded;
    box > 0: nearest periodic images; with ``ewald`` also the periodic
    images' (Ewald) correction of g and T (the jerk stays nearest-image)."""
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    m = _f64(m).ravel()
    n = x.shape[0]
    tgt = np.arange(n, dtype=np.int64) if targets is None else \
        np.ascontiguousarray(targets, dtype=np.int64)
    k = tgt.size
    acc = np.empty((k, 3))
    jerk = np.empty((k, 3))
    tid = np.empty((k, 6))
    if ewald:
        if not box > 0:
            raise ValueError("Ewald sums need a periodic box")
        _load().orc_direct_ewald(n, _ptr(x), _ptr(v), _ptr(m), float(eps), float(G), float(box), k,
                                 _ptr(tgt), _ptr(acc), _ptr(jerk), _ptr(tid))
    else:
        _load().orc_direct_box(n, _ptr(x), _ptr(v), _ptr(m), float(eps), float(G), float(box), k,
                               _ptr(tgt), _ptr(acc), _ptr(jerk), _ptr(tid))
    return acc, jerk, tid


def direct_soft(x, v, m, h, G, targets=None):
    """Direct sum with per-particle softening lengths h (n,): each pair's
    kernel is the mean of its two particles' kernels.  At particles
    ``targets`` (default: all), self excluded."""
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    m = _f64(m).ravel()
    h = _f64(h).ravel()
    n = x.shape[0]
    tgt = np.arange(n, dtype=np.int64) if targets is None else \
        np.ascontiguousarray(targets, dtype=np.int64)
    k = tgt.size
    p = np.ascontiguousarray(x[tgt])
    pv = np.ascontiguousarray(v[tgt])
    hp = np.ascontiguousarray(h[tgt])
    acc, jerk, tid = np.empty((k, 3)), np.empty((k, 3)), np.empty((k, 6))
    _load().orc_field_soft(n, _ptr(x), _ptr(v), _ptr(m), _ptr(h), float(G), k, _ptr(p), _ptr(pv), _ptr(hp),
                           _ptr(tgt), _ptr(acc), _ptr(jerk), _ptr(tid))
    return acc, jerk, tid


def neighbour_length(x, k, targets=None, chunk=256, box=0.0):
    """Distance from each target particle to its k-th nearest other particle
    (the length fully adaptive softening scales with), by brute force in
    FP64: d^2 = (dx^2 + dy^2) + dz^2 with d = x_j - x_i, then the k-th
    smallest over j != i, then its square root.  box > 0: every difference
    at its nearest image, d - box rint(d / box), each operation rounded
    once (ties at half a box to the even multiple)."""
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    tgt = np.arange(n, dtype=np.int64) if targets is None else np.asarray(targets, dtype=np.int64)
    out = np.empty(tgt.size)
    L = float(box)
    for a in range(0, tgt.size, chunk):
        t = tgt[a:a + chunk]
        dx = x[None, :, 0] - x[t, 0][:, None]
        dy = x[None, :, 1] - x[t, 1][:, None]
        dz = x[None, :, 2] - x[t, 2][:, None]
        if L > 0.0:
            dx = dx - L * np.rint(dx / L)
            dy = dy - L * np.rint(dy / L)
            dz = dz - L * np.rint(dz / L)
        d2 = dx * dx + dy * dy + dz * dz
        d2[np.arange(t.size), t] = np.inf        # not itself
        out[a:a + chunk] = np.sqrt(np.partition(d2, k - 1, axis=1)[:, k - 1])
    return out


def ewald_unit(d, L, alpha=None, nr=3, nk=4):
    """Periodic (Ewald) field of a unit mass at separations ``d`` (k x 3) in a
    cube of side L: returns g, T and the corrections dg, dT to the single
    image d (T as xx yy zz xy xz yz)."""
    d = _f64(d, (-1, 3))
    k = d.shape[0]
    g, dg = np.empty((k, 3)), np.empty((k, 3))
    T, dT = np.empty((k, 6)), np.empty((k, 6))
    a = 2.0 / L if alpha is None else float(alpha)
    _load().orc_ewald_unit(k, _ptr(d), float(L), a, int(nr), int(nk), _ptr(g), _ptr(T), _ptr(dg), _ptr(dT))
    return g, T, dg, dT


def abs_scale(x, m, eps, G, targets=None, box=0.0):
    """G sum_j m_j |f d| per target: the cancellation-free size of the sum."""
    x = _f64(x, (-1, 3))
    m = _f64(m).ravel()
    n = x.shape[0]
    tgt = np.arange(n, dtype=np.int64) if targets is None else \
        np.ascontiguousarray(targets, dtype=np.int64)
    out = np.empty(tgt.size)
    _load().orc_abs_scale_box(n, _ptr(x), _ptr(m), float(eps), float(G), float(box), tgt.size,
                              _ptr(tgt), _ptr(out))
    return out


def timestep(tidal, eta, dt_max, k_max):
    """Eq. 7 tidal timestep and its block bin for each row of ``tidal`` (n x 6)."""
    t = _f64(tidal, (-1, 6))
    n = t.shape[0]
    dt = np.empty(n)
    b = np.empty(n, dtype=np.int8)
    _load().orc_timestep(n, _ptr(t), float(eta), float(dt_max), int(k_max), _ptr(dt), _ptr(b))
    return dt, b


def select(tf_ticks, bins, step_ticks, tick_bin, q_f):
    """Eq. 3 + Eq. 4.  Returns (new tf, active mask uint8, active indices)."""
    tf = np.array(tf_ticks, dtype=np.int64, copy=True)
    b = np.ascontiguousarray(bins, dtype=np.int8)
    act = np.empty(tf.size, dtype=np.uint8)
    _load().orc_select(tf.size, _ptr(tf), _ptr(b), int(step_ticks), int(tick_bin),
                       float(q_f), _ptr(act))
    return tf, act, np.nonzero(act)[0].astype(np.int64)


def predict(a0, jerk, t0, t):
    """Eq. 6 predictor a0 + j (t - t0), row by row."""
    a0 = _f64(a0, (-1, 3))
    j = _f64(jerk, (-1, 3))
    t0 = _f64(t0).ravel()
    out = np.empty_like(a0)
    _load().orc_predict(a0.shape[0], _ptr(a0), _ptr(j), _ptr(t0), float(t), _ptr(out))
    return out


def force_log(hist_a, hist_t, hist_n, rows, acc0, t):
    """Log of past forces for the polynomial predictor (Sec. 2.2).

    For each row in ``rows``: every logged (t_k, g_k) moves one slot older
    (the oldest of the ``depth`` slots is dropped), slot 0 takes the fresh
    (t, acc0[row]) and the row's count grows by one up to ``depth``.
    ``hist_a`` (depth, n, 3), ``hist_t`` (depth, n) and ``hist_n`` (n,) are
    updated in place; slot 0 is the newest.
    """
    depth = hist_t.shape[0]
    for i in rows:
        for s in range(depth - 1, 0, -1):
            hist_a[s, i] = hist_a[s - 1, i]
            hist_t[s, i] = hist_t[s - 1, i]
        hist_a[0, i] = acc0[i]
        hist_t[0, i] = t
        hist_n[i] = min(int(hist_n[i]) + 1, depth)


def poly_nodes(hist_t, hist_n, order, i):
    """Times of the logged forces row ``i`` extrapolates from: the newest
    ones, at most ``order + 1`` of them and no more than the row has logged,
    stopping before the first slot that is not strictly older than the one
    before it (so the interpolation nodes are distinct)."""
    cnt = min(int(hist_n[i]), hist_t.shape[0])
    if cnt == 0:
        return []
    ts = [float(hist_t[0, i])]
    for k in range(1, min(cnt, order + 1)):
        if not hist_t[k, i] < ts[-1]:
            break
        ts.append(float(hist_t[k, i]))
    return ts


def predict_poly(hist_a, hist_t, hist_n, order, t):
    """Polynomial predictor (Sec. 2.2): for each row, the interpolating
    polynomial through its logged forces at the times :func:`poly_nodes`
    picks (degree ``len - 1 <= order``), evaluated at ``t`` in Lagrange form
    ``sum_k g_k prod_{m != k} (t - t_m) / (t_k - t_m)``.  Order 1 is the
    linear predictor that removes the leading time-lag error; order 0 holds
    the newest logged force.  Rows with nothing logged come back as NaN.
    Returns (n, 3)."""
    n = hist_t.shape[1]
    out = np.full((n, 3), np.nan)
    for i in range(n):
        ts = poly_nodes(hist_t, hist_n, order, i)
        if not ts:
            continue
        acc = np.zeros(3)
        for k in range(len(ts)):
            w = 1.0
            for mm in range(len(ts)):
                if mm != k:
                    w *= (t - ts[mm]) / (ts[k] - ts[mm])
            acc += w * hist_a[k, i]
        out[i] = acc
    return out


def predict_poly_weight_sum(hist_t, hist_n, order, t):
    """sum_k |Lagrange weight k| per row: the factor by which the
    predictor's rounding can grow relative to the logged forces."""
    n = hist_t.shape[1]
    out = np.zeros(n)
    for i in range(n):
        ts = poly_nodes(hist_t, hist_n, order, i)
        for k in range(len(ts)):
            w = 1.0
            for mm in range(len(ts)):
                if mm != k:
                    w *= (t - ts[mm]) / (ts[k] - ts[mm])
            out[i] += abs(w)
    return out


def adjoint(x, m, w, eps, G, k=None):
    """Exact dL/dx_k and dL/dm_k of L = sum_i w_i . a_i at particles ``k``."""
    x = _f64(x, (-1, 3))
    m = _f64(m).ravel()
    w = _f64(w, (-1, 3))
    n = x.shape[0]
    kk = np.arange(n, dtype=np.int64) if k is None else np.ascontiguousarray(k, dtype=np.int64)
    dx = np.empty((kk.size, 3))
    dm = np.empty(kk.size)
    _load().orc_adjoint(n, _ptr(x), _ptr(m), _ptr(w), float(eps), float(G), kk.size, _ptr(kk),
                        _ptr(dx), _ptr(dm))
    return dx, dm


def moments(x, v, m, idx):
    """Multipoles of the particles ``idx``: dict of M, com, u, Q, Qdot, lo, hi."""
    x = _f64(x, (-1, 3))
    v = _f64(v, (-1, 3))
    m = _f64(m).ravel()
    ii = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(25)
    _load().orc_moments(ii.size, _ptr(ii), _ptr(x), _ptr(v), _ptr(m), _ptr(out))
    return {"M": out[0], "com": out[1:4], "u": out[4:7], "Q": out[7:13], "Qdot": out[13:19],
            "lo": out[19:22], "hi": out[22:25]}


# ---- Price & Monaghan terms of fully adaptive softening --------------------
# With h_i tied to the kernel-weighted number density, h_i^3 n_i = 3 N/(4 pi),
# n_i = sum_j W(r_ij, h_i) (self included), the potential energy
#   E = (G/2) sum_i sum_{j != i} m_i m_j phi(r_ij, h_i)
# depends on the positions through the h_i too; -(1/m_i) dE/dx_i is the
# mean-kernel force plus the correction computed here (numpy, O(n^2), for
# small sets).  phi(r, h) = psi(r/h) / h is the potential of a unit mass
# spread by the cubic spline of support h, so that phi'(r)/r is the force
# kernel f of `kernel` (G = 1).

def m4_shape(u):
    """w(u), w'(u) of the cubic spline with support 1: W(r, h) = 8/(pi h^3) w(r/h)."""
    u = np.asarray(u, dtype=np.float64)
    w = np.where(u < 0.5, 1.0 - 6.0 * u**2 + 6.0 * u**3, np.where(u < 1.0, 2.0 * (1.0 - u)**3, 0.0))
    wp = np.where(u < 0.5, -12.0 * u + 18.0 * u**2, np.where(u < 1.0, -6.0 * (1.0 - u)**2, 0.0))
    return w, wp


def soft_potential(u):
    """psi(u): -1/u beyond the support; inside it the integral of u F(u)
    (F = h^3 f) from 1, added to psi(1) = -1, in closed form."""
    u = np.asarray(u, dtype=np.float64)
    with np.errstate(divide="ignore"):
        inner = 16.0 / 3 * u**2 - 48.0 / 5 * u**4 + 32.0 / 5 * u**5 - 14.0 / 5
        outer = 32.0 / 3 * u**2 - 16.0 * u**3 + 48.0 / 5 * u**4 - 32.0 / 15 * u**5 + 1.0 / (15.0 * u) - 16.0 / 5
        far = -1.0 / u
    return np.where(u < 0.5, inner, np.where(u < 1.0, outer, far))


def pm_lengths(x, n_ngb, iters=200):
    """h_i with sum_j w(r_ij / h_i) = 3 n_ngb / 32 (self included), that is
    h^3 n = 3 n_ngb / (4 pi); bisection in FP64 (the sum grows with h)."""
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    target = 3.0 * n_ngb / 32.0
    if not (1.0 < target < n):
        raise ValueError("need 32/3 < n_ngb < 32 n / 3")
    h = np.empty(n)
    for i in range(n):
        r = np.sqrt(np.sum((x - x[i])**2, axis=1))
        lo, hi = 0.0, 2.0 * r.max() + 1e-300
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:   # no double left between the ends
                break
            if m4_shape(r / mid)[0].sum() < target:
                lo = mid
            else:
                hi = mid
        h[i] = 0.5 * (lo + hi)
    return h


def pm_terms(x, m, h, n_ngb, G):
    """Per particle: Omega_i = 1 + (h/(3n)) dn/dh = -(32/(9 N)) sum_j u w'(u),
    and Z_i = (G/2) m_i h_i / (3 n_i Omega_i) sum_{j != i} m_j dphi/dh(r_ij, h_i),
    with dphi/dh = -(psi(u) + u^2 F(u)) / h^2."""
    x, m, h = _f64(x, (-1, 3)), _f64(m).ravel(), _f64(h).ravel()
    n = x.shape[0]
    C = 3.0 * n_ngb / (4.0 * np.pi)
    omega, Z = np.empty(n), np.empty(n)
    for i in range(n):
        r = np.sqrt(np.sum((x - x[i])**2, axis=1))
        u = r / h[i]
        _, wp = m4_shape(u)
        omega[i] = -(32.0 / (9.0 * n_ngb)) * np.sum(u * wp)
        f, _, _ = kernel(r, h[i])
        F = f * h[i]**3
        dphidh = -(soft_potential(u) + u * u * F) / h[i]**2
        mm = m.copy()
        mm[i] = 0.0
        ni = C / h[i]**3
        Z[i] = 0.5 * G * m[i] * h[i] / (3.0 * ni * omega[i]) * np.sum(mm * dphidh)
    return omega, Z


def pm_correction(x, m, h, n_ngb, G):
    """The extra acceleration (n, 3): -(1/m_i) sum_{j != i} [Z_i W'(r, h_i)
    + Z_j W'(r, h_j)] d / r with d = x_j - x_i and W' = dW/dr."""
    x, m, h = _f64(x, (-1, 3)), _f64(m).ravel(), _f64(h).ravel()
    _, Z = pm_terms(x, m, h, n_ngb, G)
    n = x.shape[0]
    a = np.zeros((n, 3))
    for i in range(n):
        d = x - x[i]
        r = np.sqrt(np.sum(d * d, axis=1))
        r[i] = 1.0
        wpi = m4_shape(r / h[i])[1] * 8.0 / (np.pi * h[i]**4)
        wpj = m4_shape(r / h)[1] * 8.0 / (np.pi * h**4)
        c = Z[i] * wpi + Z * wpj
        c[i] = 0.0
        a[i] = -np.sum((c / r)[:, None] * d, axis=0) / m[i]
    return a


def pm_energy(x, m, n_ngb, G):
    """E = (G/2) sum_i sum_{j != i} m_i m_j phi(r_ij, h_i) with h solved at x."""
    x, m = _f64(x, (-1, 3)), _f64(m).ravel()
    h = pm_lengths(x, n_ngb)
    E = 0.0
    for i in range(x.shape[0]):
        r = np.sqrt(np.sum((x - x[i])**2, axis=1))
        phi = soft_potential(r / h[i]) / h[i]
        phi[i] = 0.0
        E += m[i] * np.sum(m * phi)
    return 0.5 * G * E
