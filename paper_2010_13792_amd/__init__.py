"""Python binding of ``libadaptgrav.so`` (the C ABI in ``include/adaptgrav.h``).

Argument marshalling only: every method of :class:`Context` checks tensor
device, dtype, shape and contiguity, then calls the C entry point of the same
name (``ag_<name>``) with raw device pointers and the context's stream.  All
computation happens in the library's HIP kernels; there is no fallback, and
importing this module fails if the library has not been built.

PyTorch supplies device memory and streams.  Arrays follow the C layouts:
vectors ``(n, 3)`` float64, symmetric tensors ``(n, 6)`` float64 in
xx yy zz xy xz yz order, index lists int32.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads the HIP runtime first, so the library binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadaptgrav.so")

AG_OK = 0
AG_EINVAL = -1
AG_ENOMEM = -2
AG_EHIP = -3
AG_ESTATE = -4
AG_ENONFINITE = -5
AG_EDEVICE = -6
AG_FP64 = 0
AG_FP32_PAIRS = 1

ENTRY_POINTS = [
    "ag_create", "ag_destroy", "ag_set_stream", "ag_sync", "ag_stats_read", "ag_stats_reset",
    "ag_last_error", "ag_tree_build", "ag_tree_build_batched", "ag_tree_refit", "ag_tree_info",
    "ag_tree_export", "ag_grav_eval",
    "ag_grav_eval_batched", "ag_grav_direct", "ag_grav_timestep", "ag_adaptive_select",
    "ag_grav_predict", "ag_grav_backward", "ag_timing_enable", "ag_timing_read",
    "ag_kick_drift", "ag_set_option", "ag_graph_begin", "ag_graph_end", "ag_graph_replay",
    "ag_force_log", "ag_grav_predict_poly", "ag_set_periodic", "ag_set_softening",
    "ag_neighbour_lengths", "ag_set_relative_opening", "ag_pm_lengths", "ag_pm_factors", "ag_pm_correct",
    "ag_grav_eval_dev", "ag_grav_timestep_dev", "ag_grav_predict_age", "ag_pm_correct_add", "ag_force_log_dev",
    "ag_grav_direct_noalloc",
]
AG_PRED_MAX_DEPTH = 4
AG_OPT_WALK_WAVES_PER_CU = 1
AG_OPT_SMALL_NODE = 2
AG_OPT_GROUP_SPAN = 3
AG_OPT_MAC_OFFSET = 4
AG_OPT_GROUP_TARGETS = 5
AG_OPT_EWALD_OPEN = 6
AG_OPT_ADJOINT_OPEN = 7
AG_OPT_MEM_LIMIT = 8
AG_OPT_GROUP_SPLIT = 9
AG_OPT_GROUP_PACK = 10
PHASES = ["build", "groups", "walk", "direct", "step", "adjoint", "ewald", "neighbour"]


class AgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"adaptgrav error {code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("n_pp", ctypes.c_uint64), ("n_pn", ctypes.c_uint64),
                ("n_targets", ctypes.c_uint64), ("n_nodes", ctypes.c_int64),
                ("n_leaf", ctypes.c_int32), ("max_level", ctypes.c_int32),
                ("n_groups", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with __graft_entry__.build() "
                          "or python -m paper_2010_13792_amd._build")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "ag_create": [ctypes.POINTER(P), ctypes.c_int, P],
        "ag_destroy": [P], "ag_set_stream": [P, P], "ag_sync": [P],
        "ag_stats_read": [P, ctypes.POINTER(Stats)], "ag_stats_reset": [P],
        "ag_tree_build": [P, I64, P, P, P, I32],
        "ag_tree_build_batched": [P, I64, P, P, P, I32, P, I32],
        "ag_tree_refit": [P, P, P, P],
        "ag_tree_info": [P, ctypes.POINTER(I64), ctypes.POINTER(I32)],
        "ag_tree_export": [P, I64, P, P, P],
        "ag_grav_eval": [P, P, I64, D, D, D, P, P, P],
        "ag_grav_eval_batched": [P, P, I64, D, D, D, P, P, P],
        "ag_grav_eval_dev": [P, P, P, D, D, D, P, P, P, P],
        "ag_grav_timestep_dev": [P, I64, P, P, P, D, D, I32, P, P],
        "ag_grav_predict_age": [P, I64, P, P, P, P, D, P],
        "ag_pm_correct_add": [P, P, P, P, P],
        "ag_grav_direct": [P, I64, P, P, P, P, I64, D, D, ctypes.c_int, P, P, P],
        "ag_grav_direct_noalloc": [P, I64, P, P, P, P, I64, D, D, ctypes.c_int, P, P, P],
        "ag_grav_timestep": [P, I64, P, I64, P, D, D, I32, P, P],
        "ag_adaptive_select": [P, I64, P, P, I64, I32, D, P, P, P, D],
        "ag_kick_drift": [P, I64, P, P, P, D, D],
        "ag_set_option": [P, I32, I64],
        "ag_set_periodic": [P, D, I32],
        "ag_set_softening": [P, I64, P],
        "ag_neighbour_lengths": [P, I32, D, P],
        "ag_pm_lengths": [P, D, P, P],
        "ag_pm_factors": [P, D, D, P, P],
        "ag_pm_correct": [P, P, P],
        "ag_set_relative_opening": [P, D, I64, P],
        "ag_graph_begin": [P], "ag_graph_end": [P], "ag_graph_replay": [P],
        "ag_grav_predict": [P, I64, P, P, P, P, D, P],
        "ag_force_log": [P, I64, P, I64, I32, P, D, P, P, P],
        "ag_force_log_dev": [P, I64, P, P, I32, P, D, P, P, P],
        "ag_grav_predict_poly": [P, I64, P, I32, I32, P, P, P, D, P],
        "ag_grav_backward": [P, P, I64, P, D, D, D, P, P],
        "ag_timing_enable": [P, ctypes.c_int],
        "ag_timing_read": [P, P, P, ctypes.c_int],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ag_last_error.argtypes = []
    lib.ag_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(code):
    if code != AG_OK:
        raise AgError(code, _lib.ag_last_error().decode())


def _ptr(t, dtype, shape_tail=None, name="array", n=None):
    """Device pointer of a contiguous CUDA/HIP tensor after checking it."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape (n, {', '.join(map(str, shape_tail))})")
    if n is not None and t.shape[0] < n:
        raise ValueError(f"{name} has {t.shape[0]} rows, needs {n}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """An ``ag_ctx``: one device, one stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        lib = load_library()
        self.device = device
        self._stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        _check(lib.ag_create(ctypes.byref(h), device, ctypes.c_void_p(self._stream.cuda_stream)))
        self._h = h
        self.n = None

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _lib.ag_destroy(self._h)
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

    @property
    def stream(self) -> torch.cuda.Stream:
        """The torch stream the context's calls are ordered on."""
        return self._stream

    def set_stream(self, stream: torch.cuda.Stream):
        self._stream = stream
        _check(_lib.ag_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def sync(self):
        _check(_lib.ag_sync(self._h))

    def stats_read(self) -> dict:
        s = Stats()
        _check(_lib.ag_stats_read(self._h, ctypes.byref(s)))
        return s.as_dict()

    def stats_reset(self):
        _check(_lib.ag_stats_reset(self._h))

    def timing_enable(self, on: bool = True):
        _check(_lib.ag_timing_enable(self._h, 1 if on else 0))

    def timing_read(self, reset: bool = True) -> dict:
        """Accumulated GPU milliseconds and launch counts per phase."""
        ms = (ctypes.c_double * len(PHASES))()
        cnt = (ctypes.c_int64 * len(PHASES))()
        _check(_lib.ag_timing_read(self._h, ctypes.cast(ms, ctypes.c_void_p),
                                   ctypes.cast(cnt, ctypes.c_void_p), 1 if reset else 0))
        return {p: {"ms": ms[k], "launches": cnt[k]} for k, p in enumerate(PHASES)}

    # -- tree ---------------------------------------------------------------
    def tree_build(self, x, v, m, n_leaf: int = 16):
        n = x.shape[0]
        _check(_lib.ag_tree_build(self._h, n, _ptr(x, torch.float64, (3,), "x"),
                                  _ptr(v, torch.float64, (3,), "v", n),
                                  _ptr(m, torch.float64, None, "m", n), int(n_leaf)))
        self.n = n

    def tree_build_batched(self, x, v, m, sys_offsets, n_leaf: int = 16):
        n = x.shape[0]
        n_sys = sys_offsets.shape[0] - 1
        _check(_lib.ag_tree_build_batched(self._h, n, _ptr(x, torch.float64, (3,), "x"),
                                          _ptr(v, torch.float64, (3,), "v", n),
                                          _ptr(m, torch.float64, None, "m", n), int(n_sys),
                                          _ptr(sys_offsets, torch.int64, None, "sys_offsets"),
                                          int(n_leaf)))
        self.n = n

    def tree_refit(self, x, v, m):
        _check(_lib.ag_tree_refit(self._h, _ptr(x, torch.float64, (3,), "x", self.n),
                                  _ptr(v, torch.float64, (3,), "v", self.n),
                                  _ptr(m, torch.float64, None, "m", self.n)))

    def tree_info(self):
        nn = ctypes.c_int64()
        ml = ctypes.c_int32()
        _check(_lib.ag_tree_info(self._h, ctypes.byref(nn), ctypes.byref(ml)))
        return int(nn.value), int(ml.value)

    def tree_export(self):
        """Copy the tree to new device tensors: (link (nn,4) int32,
        moments (nn,25) float64, perm (n,) int32)."""
        nn, _ = self.tree_info()
        dev = torch.device("cuda", self.device)
        link = torch.empty((nn, 4), dtype=torch.int32, device=dev)
        mom = torch.empty((nn, 25), dtype=torch.float64, device=dev)
        perm = torch.empty((self.n,), dtype=torch.int32, device=dev)
        _check(_lib.ag_tree_export(self._h, nn, _ptr(link, torch.int32, (4,), "link"),
                                   _ptr(mom, torch.float64, (25,), "moments"),
                                   _ptr(perm, torch.int32, None, "perm")))
        self.sync()
        return link, mom, perm

    # -- gravity ------------------------------------------------------------
    def grav_eval(self, active_idx, theta, eps, G, acc, jerk, tidal, batched=False):
        n = self.n
        k = n if active_idx is None else active_idx.shape[0]
        fn = _lib.ag_grav_eval_batched if batched else _lib.ag_grav_eval
        _check(fn(self._h, _ptr(active_idx, torch.int32, None, "active_idx"), k, float(theta),
                  float(eps), float(G), _ptr(acc, torch.float64, (3,), "acc", n),
                  _ptr(jerk, torch.float64, (3,), "jerk", n),
                  _ptr(tidal, torch.float64, (6,), "tidal", n)))

    def grav_eval_dev(self, active_idx, n_active_dev, theta, eps, G, acc, jerk, tidal, n_total=None):
        """Tree gravity at rows active_idx[:n_active_dev[0]], the count read
        on the device (no host synchronisation); n_total (int64 (1,)) gains
        the count."""
        n = self.n
        _check(_lib.ag_grav_eval_dev(self._h, _ptr(active_idx, torch.int32, None, "active_idx", n),
                                     _ptr(n_active_dev, torch.int64, None, "n_active_dev", 1), float(theta),
                                     float(eps), float(G), _ptr(acc, torch.float64, (3,), "acc", n),
                                     _ptr(jerk, torch.float64, (3,), "jerk", n),
                                     _ptr(tidal, torch.float64, (6,), "tidal", n),
                                     _ptr(n_total, torch.int64, None, "n_total", 1)))

    def grav_eval_batched(self, active_idx, theta, eps, G, acc, jerk, tidal):
        self.grav_eval(active_idx, theta, eps, G, acc, jerk, tidal, batched=True)

    def grav_direct(self, x, v, m, active_idx, eps, G, acc, jerk, tidal, precision=AG_FP64, noalloc=False):
        """Direct summation; ``noalloc`` calls ag_grav_direct_noalloc (no
        device allocation; library-held scratch shared per device)."""
        n = x.shape[0]
        k = n if active_idx is None else active_idx.shape[0]
        fn = _lib.ag_grav_direct_noalloc if noalloc else _lib.ag_grav_direct
        _check(fn(self._h, n, _ptr(x, torch.float64, (3,), "x"),
                                   _ptr(v, torch.float64, (3,), "v", n),
                                   _ptr(m, torch.float64, None, "m", n),
                                   _ptr(active_idx, torch.int32, None, "active_idx"), k,
                                   float(eps), float(G), int(precision),
                                   _ptr(acc, torch.float64, (3,), "acc", n),
                                   _ptr(jerk, torch.float64, (3,), "jerk", n),
                                   _ptr(tidal, torch.float64, (6,), "tidal", n)))

    def grav_timestep(self, tidal, eta, dt_max, k_max, dt_grav, bins, idx=None):
        n = tidal.shape[0]
        k = n if idx is None else idx.shape[0]
        _check(_lib.ag_grav_timestep(self._h, n, _ptr(idx, torch.int32, None, "idx"), k,
                                     _ptr(tidal, torch.float64, (6,), "tidal"), float(eta),
                                     float(dt_max), int(k_max),
                                     _ptr(dt_grav, torch.float64, None, "dt_grav", n),
                                     _ptr(bins, torch.int8, None, "bin", n)))

    def grav_timestep_dev(self, tidal, eta, dt_max, k_max, dt_grav, bins, idx, n_idx_dev):
        """Eq. 7 timestep and bin at rows idx[:n_idx_dev[0]] (count on the device)."""
        n = tidal.shape[0]
        _check(_lib.ag_grav_timestep_dev(self._h, n, _ptr(idx, torch.int32, None, "idx", n),
                                         _ptr(n_idx_dev, torch.int64, None, "n_idx_dev", 1),
                                         _ptr(tidal, torch.float64, (6,), "tidal"), float(eta),
                                         float(dt_max), int(k_max),
                                         _ptr(dt_grav, torch.float64, None, "dt_grav", n),
                                         _ptr(bins, torch.int8, None, "bin", n)))

    def adaptive_select(self, tf_ticks, bins, step_ticks, tick_bin, q_f, active_idx, n_active_dev,
                        t0=None, t=0.0):
        n = tf_ticks.shape[0]
        _check(_lib.ag_adaptive_select(self._h, n, _ptr(tf_ticks, torch.int64, None, "tf_ticks"),
                                       _ptr(bins, torch.int8, None, "bin", n), int(step_ticks),
                                       int(tick_bin), float(q_f),
                                       _ptr(active_idx, torch.int32, None, "active_idx", n),
                                       _ptr(n_active_dev, torch.int64, None, "n_active", 1),
                                       _ptr(t0, torch.float64, None, "t0", n), float(t)))

    def kick_drift(self, x, v, acc, dt_kick, dt_drift):
        n = x.shape[0]
        _check(_lib.ag_kick_drift(self._h, n, _ptr(x, torch.float64, (3,), "x"),
                                  _ptr(v, torch.float64, (3,), "v", n),
                                  _ptr(acc, torch.float64, (3,), "acc", n), float(dt_kick),
                                  float(dt_drift)))

    def set_option(self, option: int, value: int):
        _check(_lib.ag_set_option(self._h, int(option), int(value)))

    def graph_begin(self):
        _check(_lib.ag_graph_begin(self._h))

    def graph_end(self):
        _check(_lib.ag_graph_end(self._h))

    def graph_replay(self):
        _check(_lib.ag_graph_replay(self._h))

    def grav_predict(self, acc0, jerk, t0, t, acc_out, mask=None):
        n = acc0.shape[0]
        _check(_lib.ag_grav_predict(self._h, n, _ptr(mask, torch.uint8, None, "mask", n),
                                    _ptr(acc0, torch.float64, (3,), "acc0"),
                                    _ptr(jerk, torch.float64, (3,), "jerk", n),
                                    _ptr(t0, torch.float64, None, "t0", n), float(t),
                                    _ptr(acc_out, torch.float64, (3,), "acc_out", n)))

    def grav_predict_age(self, acc0, jerk, age_ticks, tick, acc_out, mask=None):
        """Eq. 6 with t - t0 = age_ticks * tick (the Eq. 3 force-age counters)."""
        n = acc0.shape[0]
        _check(_lib.ag_grav_predict_age(self._h, n, _ptr(mask, torch.uint8, None, "mask", n),
                                        _ptr(acc0, torch.float64, (3,), "acc0"),
                                        _ptr(jerk, torch.float64, (3,), "jerk", n),
                                        _ptr(age_ticks, torch.int64, None, "age_ticks", n), float(tick),
                                        _ptr(acc_out, torch.float64, (3,), "acc_out", n)))

    def set_softening(self, h=None):
        """Per-particle softening lengths (device float64 (n,)); None clears."""
        if h is None:
            _check(_lib.ag_set_softening(self._h, 0, None))
            return
        _check(_lib.ag_set_softening(self._h, h.shape[0], _ptr(h, torch.float64, None, "h")))

    def set_relative_opening(self, alpha: float = 0.0, acc=None):
        """Relative opening test with tolerance ``alpha`` against the sizes of
        ``acc`` (device float64 (n, 3), the previous accelerations); alpha = 0
        or acc = None turns it off."""
        if acc is None or alpha == 0.0:
            _check(_lib.ag_set_relative_opening(self._h, float(alpha), 0, None))
            return
        _check(_lib.ag_set_relative_opening(self._h, float(alpha), acc.shape[0],
                                            _ptr(acc, torch.float64, (3,), "acc")))

    def neighbour_lengths(self, k: int, out=None, scale: float = 1.0):
        """Distance of every particle to its k-th nearest other particle, times
        ``scale``, from the built tree (device float64 (n,), input order)."""
        n = self.n
        if out is None:
            if n is None:
                raise AgError(AG_ESTATE, "neighbour lengths before a tree build")
            out = torch.empty(n, dtype=torch.float64, device=torch.device("cuda", self.device))
        _check(_lib.ag_neighbour_lengths(self._h, int(k), float(scale), _ptr(out, torch.float64, None, "out", n)))
        return out

    def _pm_out(self, out, shape, name):
        n = self.n
        if out is None:
            if n is None:
                raise AgError(AG_ESTATE, "Price & Monaghan terms before a tree build")
            out = torch.empty((n,) + shape, dtype=torch.float64, device=torch.device("cuda", self.device))
        return out, _ptr(out, torch.float64, shape or None, name, n)

    def pm_lengths(self, n_ngb: float, h=None, omega=None):
        """Price & Monaghan lengths h and Omega from the built tree (device
        float64 (n,) each, input order); synchronises."""
        h, ph = self._pm_out(h, (), "h")
        omega, po = self._pm_out(omega, (), "omega")
        _check(_lib.ag_pm_lengths(self._h, float(n_ngb), ph, po))
        return h, omega

    def pm_factors(self, n_ngb: float, G: float, omega, z=None):
        """The correction's factors Z (n,), with the softening lengths the
        tree was built with and Omega from pm_lengths."""
        z, pz = self._pm_out(z, (), "z")
        _check(_lib.ag_pm_factors(self._h, float(n_ngb), float(G),
                                  _ptr(omega, torch.float64, None, "omega", self.n), pz))
        return z

    def pm_correct(self, z, out=None):
        """The correction's acceleration (n, 3) from the factors Z."""
        out, pa = self._pm_out(out, (3,), "out")
        _check(_lib.ag_pm_correct(self._h, _ptr(z, torch.float64, None, "z", self.n), pa))
        return out

    def pm_correct_add(self, z, acc, idx=None, n_idx_dev=None):
        """Add the correction's acceleration to acc (n, 3) at rows
        idx[:n_idx_dev[0]] (count on the device), or at every row."""
        if (idx is None) != (n_idx_dev is None):
            raise ValueError("idx and n_idx_dev go together")
        _check(_lib.ag_pm_correct_add(self._h, _ptr(z, torch.float64, None, "z", self.n),
                                      _ptr(idx, torch.int32, None, "idx"),
                                      _ptr(n_idx_dev, torch.int64, None, "n_idx_dev", 1),
                                      _ptr(acc, torch.float64, (3,), "acc", self.n)))

    def set_periodic(self, box: float, ewald: bool = False):
        """Periodic cube of side ``box`` (0: open): nearest-image pairs, or
        with ``ewald`` the full periodic g and T (j stays nearest-image)."""
        _check(_lib.ag_set_periodic(self._h, float(box), 1 if ewald else 0))

    @staticmethod
    def _log_ptrs(hist_a, hist_t, hist_n):
        """Checked pointers of a force log: hist_a (depth, n, 3), hist_t
        (depth, n), hist_n (n,)."""
        if hist_a.dim() != 3 or hist_a.shape[2] != 3:
            raise ValueError("hist_a must have shape (depth, n, 3)")
        depth, n = hist_a.shape[0], hist_a.shape[1]
        if tuple(hist_t.shape) != (depth, n) or tuple(hist_n.shape) != (n,):
            raise ValueError("hist_t must be (depth, n) and hist_n (n,) for hist_a (depth, n, 3)")
        return (depth, n, _ptr(hist_a, torch.float64, None, "hist_a"),
                _ptr(hist_t, torch.float64, None, "hist_t"), _ptr(hist_n, torch.int32, None, "hist_n"))

    def force_log(self, acc0, t, hist_a, hist_t, hist_n, idx=None):
        depth, n, pa, pt, pn = self._log_ptrs(hist_a, hist_t, hist_n)
        k = n if idx is None else idx.shape[0]
        _check(_lib.ag_force_log(self._h, n, _ptr(idx, torch.int32, None, "idx"), k, depth,
                                 _ptr(acc0, torch.float64, (3,), "acc0", n), float(t), pa, pt, pn))

    def force_log_dev(self, acc0, t, hist_a, hist_t, hist_n, idx, n_idx_dev):
        """force_log at rows idx[:n_idx_dev[0]] (count on the device)."""
        depth, n, pa, pt, pn = self._log_ptrs(hist_a, hist_t, hist_n)
        _check(_lib.ag_force_log_dev(self._h, n, _ptr(idx, torch.int32, None, "idx", n),
                                     _ptr(n_idx_dev, torch.int64, None, "n_idx_dev", 1), depth,
                                     _ptr(acc0, torch.float64, (3,), "acc0", n), float(t), pa, pt, pn))

    def grav_predict_poly(self, hist_a, hist_t, hist_n, order, t, acc_out, mask=None):
        depth, n, pa, pt, pn = self._log_ptrs(hist_a, hist_t, hist_n)
        _check(_lib.ag_grav_predict_poly(self._h, n, _ptr(mask, torch.uint8, None, "mask", n), depth,
                                         int(order), pa, pt, pn, float(t),
                                         _ptr(acc_out, torch.float64, (3,), "acc_out", n)))

    def grav_backward(self, active_idx, w, theta, eps, G, dLdx, dLdm):
        n = self.n
        k = n if active_idx is None else active_idx.shape[0]
        _check(_lib.ag_grav_backward(self._h, _ptr(active_idx, torch.int32, None, "active_idx"), k,
                                     _ptr(w, torch.float64, (3,), "w", n), float(theta), float(eps),
                                     float(G), _ptr(dLdx, torch.float64, (3,), "dLdx", n),
                                     _ptr(dLdm, torch.float64, None, "dLdm", n)))


from .autograd import GravEval, grav_eval  # noqa: E402,F401
