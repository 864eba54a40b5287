"""ctypes binding of libxsec.so: argument marshalling only.

Tensors passed in must already live on the GPU (torch is used for device memory
and streams); every computation happens in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libxsec.so"

PROFILES = {"doppler": 0, "gauss_fixed": 1, "lorentz": 2, "voigt": 3, "gh_sampled": 4, "gh_binned": 5,
            "vvoigt": 6, "vvoigt_norm": 7, "doppler_binned": 8, "lorentz_binned": 9, "superlines": 10}
PRECISIONS = {"fp64": 0, "fp32": 1}
BROADENING = {"const": 0, "per_line": 1, "a0_jlower": 2}
STATUS = {0: "XS_OK", 1: "XS_ERR_ARG", 2: "XS_ERR_INDEX", 3: "XS_ERR_NU_NONPOS", 4: "XS_ERR_HIP",
          5: "XS_ERR_OOM", 6: "XS_ERR_STATE", 7: "XS_ERR_UNSUPPORTED", 8: "XS_ERR_INJECTED"}


class XsecError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class XsOpts(ctypes.Structure):
    _fields_ = [
        ("nu_a", ctypes.c_double), ("nu_b", ctypes.c_double), ("n_points", ctypes.c_int64),
        ("cutoff", ctypes.c_double), ("mass_da", ctypes.c_double), ("T0", ctypes.c_double),
        ("P0", ctypes.c_double), ("profile", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("broadening", ctypes.c_int32), ("index_base", ctypes.c_int32),
        ("alpha_fixed", ctypes.c_double), ("gamma_const", ctypes.c_double), ("n_const", ctypes.c_double),
        ("slices_per_wave", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
        ("a_is_log", ctypes.c_int32), ("n_split", ctypes.c_int32), ("tp_block", ctypes.c_int32),
        ("vv_beta", ctypes.c_int32), ("vv_radius", ctypes.c_double), ("gh_nodes", ctypes.c_int32),
    ]


class XsKernelTimes(ctypes.Structure):
    _fields_ = [("forward_ms", ctypes.c_double), ("core_ms", ctypes.c_double), ("prep_ms", ctypes.c_double),
                ("forward_launches", ctypes.c_int64), ("core_launches", ctypes.c_int64),
                ("prep_launches", ctypes.c_int64), ("combine_ms", ctypes.c_double),
                ("combine_launches", ctypes.c_int64), ("forward_tp", ctypes.c_int64),
                ("far_ms", ctypes.c_double), ("far_launches", ctypes.c_int64)]


_lib = None


def lib_path() -> str:
    return os.path.join(HERE, _LIB_NAME)


def load_library() -> ctypes.CDLL:
    """Load the in-tree libxsec.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1801_09803_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "xs_opts_default": (i32, [ctypes.POINTER(XsOpts)]),
        "xs_plan_create": (i32, [ctypes.POINTER(XsOpts), ctypes.POINTER(P)]),
        "xs_plan_destroy": (i32, [P]),
        "xs_set_states": (i32, [P, i64, P, P, P, P]),
        "xs_set_broadening_table": (i32, [P, i32, P, P]),
        "xs_set_lines": (i32, [P, i64, P, P, P, P, P, P]),
        "xs_set_intensity_threshold": (i32, [P, i32, dbl, dbl]),
        "xs_lines_kept": (i32, [P, ctypes.POINTER(i64)]),
        "xs_partition_function": (i32, [P, i32, P, P, P, P]),
        "xs_set_intensity_kind": (i32, [P, i32]),
        "xs_set_vibrational_labels": (i32, [P, i32, P, P]),
        "xs_cross_section_nlte": (i32, [P, i32, P, P, P, P, P]),
        "xs_partition_function_nlte": (i32, [P, i32, P, P, P, P]),
        "xs_partition_moments": (i32, [P, i32, P, P, P, P, P, P]),
        "xs_lifetimes": (i32, [P, i64, P, P, P, P]),
        "xs_cooling_function": (i32, [P, i64, P, P, P, i32, P, P, P]),
        "xs_cross_section": (i32, [P, i32, P, P, P, P]),
        "xs_cross_section_adjoint": (i32, [P, dbl, dbl, P, P, P, P, P, P, P]),
        "xs_graph_create": (i32, [P, i32, P, P, P, ctypes.POINTER(P)]),
        "xs_graph_set_tp": (i32, [P, P, P, P]),
        "xs_graph_launch": (i32, [P, P]),
        "xs_graph_destroy": (i32, [P]),
        "xs_graph_workspace_bytes": (ctypes.c_size_t, [P]),
        "xs_stream_begin": (i32, [P, i32, P, P, P, P, ctypes.POINTER(P)]),
        "xs_stream_chunk": (i32, [P, i64, P, P, P, P, P]),
        "xs_stream_chunk_device": (i32, [P, i64, P, P, P, P, P]),
        "xs_stream_end": (i32, [P, ctypes.POINTER(i64)]),
        "xs_stream_checkpoint": (i32, [P, ctypes.c_char_p]),
        "xs_stream_resume": (i32, [P, ctypes.c_char_p, P, P, ctypes.POINTER(P)]),
        "xs_stream_stats": (i32, [P, ctypes.POINTER(i64)]),
        "xs_set_tile_config": (i32, [P, i32, i32, i32, i32]),
        "xs_get_tile_config": (i32, [P, ctypes.POINTER(i32)]),
        "xs_autotune": (i32, [P, i32, P, P, dbl, P, ctypes.POINTER(i32)]),
        "xs_set_timing": (i32, [P, i32]),
        "xs_kernel_times": (i32, [P, ctypes.POINTER(XsKernelTimes)]),
        "xs_valu_probe": (i32, [P, i64, i32, P]),
        "xs_workspace_bytes": (ctypes.c_size_t, [P]),
        "xs_last_error": (ctypes.c_char_p, []),
        "xs_version": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def valu_probe(out, iters: int):
    """xs_valu_probe on the float32 device tensor out (one value per thread), on torch's
    current stream."""
    import torch
    if not out.is_cuda or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 CUDA tensor")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _check(load_library().xs_valu_probe(ctypes.c_void_p(out.data_ptr()), out.numel(), int(iters), stream))


def abi_version() -> int:
    return int(load_library().xs_version())


def _check(status: int):
    if status != 0:
        msg = load_library().xs_last_error()
        raise XsecError(status, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _owner(obj) -> bool:
    """True in the process that created obj's library handle."""
    return getattr(obj, "_pid", None) == os.getpid()


def _same_length(what: str, *named):
    """Raise ValueError unless every given (name, tensor) pair has the same number of
    elements (None entries are skipped); returns that number."""
    n = None
    for name, t in named:
        if t is None:
            continue
        if n is None:
            n, first = t.numel(), name
        elif t.numel() != n:
            raise ValueError(f"{what}: {name} has {t.numel()} values, {first} has {n}")
    return 0 if n is None else n


def _host_doubles(vals: Sequence[float]):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


class Plan:
    """One grid + profile configuration; owns the library plan and its workspace."""

    def __init__(self, nu_a: float, nu_b: float, n_points: int, mass_da: float, *,
                 cutoff: float = 25.0, profile: str = "voigt", precision: str = "fp32",
                 broadening: str = "per_line", T0: float = 296.0, P0: float = 1.0,
                 index_base: int = 0, alpha_fixed: float = 0.0, gamma_const: float = 0.0,
                 n_const: float = 0.0, slices_per_wave: int = 0, waves_per_block: int = 0,
                 a_is_log: bool = False, n_split: int = 0, tp_block: int = 0,
                 vv_radius: float = 0.0, vv_beta: bool = False, gh_nodes: int = 0):
        import torch
        self._torch = torch
        lib = load_library()
        o = XsOpts()
        _check(lib.xs_opts_default(ctypes.byref(o)))
        o.nu_a, o.nu_b, o.n_points = float(nu_a), float(nu_b), int(n_points)
        o.cutoff, o.mass_da, o.T0, o.P0 = float(cutoff), float(mass_da), float(T0), float(P0)
        o.profile = PROFILES[profile]
        o.precision = PRECISIONS[precision]
        o.broadening = BROADENING[broadening]
        o.index_base = int(index_base)
        o.alpha_fixed, o.gamma_const, o.n_const = float(alpha_fixed), float(gamma_const), float(n_const)
        o.slices_per_wave = int(slices_per_wave)
        o.waves_per_block = int(waves_per_block)
        o.a_is_log = 1 if a_is_log else 0
        o.n_split = int(n_split)
        o.tp_block = int(tp_block)
        o.vv_radius = float(vv_radius)
        o.vv_beta = 1 if vv_beta else 0
        o.gh_nodes = int(gh_nodes)
        h = ctypes.c_void_p()
        _check(lib.xs_plan_create(ctypes.byref(o), ctypes.byref(h)))
        self._lib = lib
        self._h = h
        self._pid = os.getpid()
        self.opts = o
        self.n_points = int(n_points)
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64

    # -- helpers
    def _stream(self):
        return ctypes.c_void_p(self._torch.cuda.current_stream().cuda_stream)

    def _dev(self, t, dtype, name):
        if t is None:
            return None
        if not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def close(self):
        # a process forked after the GPU was initialised (e.g. a multiprocessing worker)
        # inherits this object but must not call into the HIP runtime
        if getattr(self, "_h", None) is not None and self._h.value and _owner(self):
            self._lib.xs_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- ABI calls
    def set_states(self, E, g, J=None):
        torch = self._torch
        E = self._dev(E, torch.float64, "E")
        g = self._dev(g, torch.int32, "g")
        J = self._dev(J, torch.int32, "J")
        n = _same_length("set_states", ("E", E), ("g", g), ("J", J))
        self._states = (E, g, J)
        self._n_lines = None   # the library drops the line set with new states
        _check(self._lib.xs_set_states(self._h, n, _ptr(E), _ptr(g), _ptr(J), self._stream()))

    def set_broadening_table(self, gamma_ref, n_exp):
        import numpy as np
        gr = np.ascontiguousarray(np.asarray(gamma_ref, dtype=np.float32))
        ne = np.ascontiguousarray(np.asarray(n_exp, dtype=np.float32))
        if gr.shape != ne.shape:
            raise ValueError("table arrays differ in length")
        _check(self._lib.xs_set_broadening_table(self._h, gr.size, gr.ctypes.data, ne.ctypes.data))

    def set_lines(self, upper, lower, A, gamma_ref=None, n_exp=None):
        torch = self._torch
        upper = self._dev(upper, torch.int32, "upper")
        lower = self._dev(lower, torch.int32, "lower")
        A = self._dev(A, torch.float32, "A")
        gamma_ref = self._dev(gamma_ref, torch.float32, "gamma_ref")
        n_exp = self._dev(n_exp, torch.float32, "n_exp")
        n = _same_length("set_lines", ("upper", upper), ("lower", lower), ("A", A), ("gamma_ref", gamma_ref),
                         ("n_exp", n_exp))
        self._n_lines = None
        _check(self._lib.xs_set_lines(self._h, n, _ptr(upper), _ptr(lower), _ptr(A),
                                      _ptr(gamma_ref), _ptr(n_exp), self._stream()))
        self._n_lines = n

    def n_lines(self) -> int:
        """Transitions given to the last set_lines (the length of the per-line gradients)."""
        n = getattr(self, "_n_lines", None)
        if n is None:
            raise ValueError("no line set: call set_lines first")
        return n

    def lines_kept(self) -> int:
        n = ctypes.c_int64()
        _check(self._lib.xs_lines_kept(self._h, ctypes.byref(n)))
        return int(n.value)

    def partition_function(self, T: Sequence[float]):
        torch = self._torch
        T = list(T)
        Q = torch.empty(len(T), dtype=torch.float64, device="cuda")
        dQ = torch.empty(len(T), dtype=torch.float64, device="cuda")
        _check(self._lib.xs_partition_function(self._h, len(T), _host_doubles(T), _ptr(Q), _ptr(dQ),
                                               self._stream()))
        return Q, dQ

    def partition_moments(self, T: Sequence[float]):
        """(Q, Q' = T dQ/dT, Q'' = sum g x^2 e^-x, C_p in J/K/mol) per temperature."""
        torch = self._torch
        T = list(T)
        out = [torch.empty(len(T), dtype=torch.float64, device="cuda") for _ in range(4)]
        _check(self._lib.xs_partition_moments(self._h, len(T), _host_doubles(T), *[_ptr(x) for x in out],
                                              self._stream()))
        return tuple(out)

    def lifetimes(self, upper, A):
        """Radiative lifetime (s) of every state of the plan: 1 / sum of A leaving it."""
        torch = self._torch
        upper = self._dev(upper, torch.int32, "upper")
        A = self._dev(A, torch.float32, "A")
        n = _same_length("lifetimes", ("upper", upper), ("A", A))
        states = getattr(self, "_states", None)
        if states is None:
            raise ValueError("set_states must come first")
        tau = torch.empty(states[0].numel(), dtype=torch.float64, device="cuda")
        _check(self._lib.xs_lifetimes(self._h, n, _ptr(upper), _ptr(A), _ptr(tau), self._stream()))
        return tau

    def cooling_function(self, upper, lower, A, T: Sequence[float]):
        """W(T) (erg/s/sr/molecule) of the given transitions at each temperature."""
        torch = self._torch
        upper = self._dev(upper, torch.int32, "upper")
        lower = self._dev(lower, torch.int32, "lower")
        A = self._dev(A, torch.float32, "A")
        n = _same_length("cooling_function", ("upper", upper), ("lower", lower), ("A", A))
        T = list(T)
        W = torch.empty(len(T), dtype=torch.float64, device="cuda")
        _check(self._lib.xs_cooling_function(self._h, n, _ptr(upper), _ptr(lower), _ptr(A), len(T),
                                             _host_doubles(T), _ptr(W), self._stream()))
        return W

    def set_vibrational_labels(self, labels, n_labels: Optional[int] = None):
        """Non-LTE: per-state vibrational manifold labels (None returns to LTE); the line
        set must be set again afterwards."""
        torch = self._torch
        if labels is None:
            self._n_lines = None
            _check(self._lib.xs_set_vibrational_labels(self._h, 0, None, self._stream()))
            return
        labels = self._dev(labels, torch.int32, "labels")
        states = getattr(self, "_states", None)
        if states is None:
            raise ValueError("set_states must come first")
        if labels.numel() != states[0].numel():
            raise ValueError(f"labels has {labels.numel()} values for {states[0].numel()} states")
        if n_labels is None:
            n_labels = int(labels.max().item()) + 1 if labels.numel() else 1
        self._labels = labels
        self._n_lines = None   # the library drops the line set with new labels
        _check(self._lib.xs_set_vibrational_labels(self._h, int(n_labels), _ptr(labels), self._stream()))

    def cross_section_nlte(self, T_rot: Sequence[float], T_vib: Sequence[float], P: Sequence[float], out=None):
        """Cross sections with two-temperature populations at (T_rot, T_vib, P) points."""
        torch = self._torch
        T_rot, T_vib, P = list(T_rot), list(T_vib), list(P)
        if not (len(T_rot) == len(T_vib) == len(P)):
            raise ValueError("T_rot, T_vib and P differ in length")
        if out is None:
            out = torch.empty((len(P), self.n_points), dtype=self.dtype, device="cuda")
        else:
            out = self._dev(out, self.dtype, "out")
            if out.numel() != len(P) * self.n_points:
                raise ValueError("out has the wrong size")
        _check(self._lib.xs_cross_section_nlte(self._h, len(P), _host_doubles(T_rot), _host_doubles(T_vib),
                                               _host_doubles(P), _ptr(out), self._stream()))
        return out

    def partition_function_nlte(self, T_rot: Sequence[float], T_vib: Sequence[float]):
        torch = self._torch
        T_rot, T_vib = list(T_rot), list(T_vib)
        if len(T_rot) != len(T_vib):
            raise ValueError("T_rot and T_vib differ in length")
        Q = torch.empty(len(T_rot), dtype=torch.float64, device="cuda")
        _check(self._lib.xs_partition_function_nlte(self._h, len(T_rot), _host_doubles(T_rot), _host_doubles(T_vib),
                                                    _ptr(Q), self._stream()))
        return Q

    def set_intensity_kind(self, kind: str = "absorption"):
        """Cross sections of absorption intensities (Eq. 1) or of emissivities ("emission")."""
        kinds = {"absorption": 0, "emission": 1}
        _check(self._lib.xs_set_intensity_kind(self._h, kinds[kind]))

    def cross_section(self, T: Sequence[float], P: Sequence[float], out=None):
        torch = self._torch
        T, P = list(T), list(P)
        if len(T) != len(P):
            raise ValueError("T and P differ in length")
        if out is None:
            out = torch.empty((len(T), self.n_points), dtype=self.dtype, device="cuda")
        else:
            out = self._dev(out, self.dtype, "out")
            if out.numel() != len(T) * self.n_points:
                raise ValueError("out has the wrong size")
        _check(self._lib.xs_cross_section(self._h, len(T), _host_doubles(T), _host_doubles(P), _ptr(out),
                                          self._stream()))
        return out

    def cross_section_adjoint(self, T: float, P: float, grad_sigma, n_lines: Optional[int] = None,
                              want_broadening: bool = True):
        """Returns (dL/dT, dL/dP, dL/dlnA, dL/dgamma_ref, dL/dn) as device tensors; the
        per-line gradients have one value per transition of the last set_lines (n_lines, if
        given, must equal that count)."""
        torch = self._torch
        n_set = self.n_lines()
        if n_lines is not None and int(n_lines) != n_set:
            raise ValueError(f"n_lines = {n_lines}, but the line set has {n_set} transitions")
        n_lines = n_set
        grad_sigma = self._dev(grad_sigma, self.dtype, "grad_sigma")
        if grad_sigma.numel() != self.n_points:
            raise ValueError("grad_sigma must have n_points values")
        dT = torch.empty(1, dtype=torch.float64, device="cuda")
        dP = torch.empty(1, dtype=torch.float64, device="cuda")
        # per-line gradients are double for both precisions (their values lie far below
        # the float range for cross sections in cm^2/molecule)
        dlnA = torch.empty(n_lines, dtype=torch.float64, device="cuda")
        dg = torch.empty(n_lines, dtype=torch.float64, device="cuda") if want_broadening else None
        dn = torch.empty(n_lines, dtype=torch.float64, device="cuda") if want_broadening else None
        _check(self._lib.xs_cross_section_adjoint(self._h, float(T), float(P), _ptr(grad_sigma), _ptr(dT),
                                                  _ptr(dP), _ptr(dlnA), _ptr(dg), _ptr(dn), self._stream()))
        return dT, dP, dlnA, dg, dn

    def set_intensity_threshold(self, mode: str = "none", i_crit: float = 1e-29, nu_crit: float = 2000.0):
        """Intensity threshold: "none", "constant" (I >= i_crit) or "hitran" (dynamic cut-off)."""
        modes = {"none": 0, "constant": 1, "hitran": 2}
        _check(self._lib.xs_set_intensity_threshold(self._h, modes[mode], float(i_crit), float(nu_crit)))

    def set_tile_config(self, waves: int = 0, slices: int = 0, n_split: int = 0, tp_block: int = 0):
        _check(self._lib.xs_set_tile_config(self._h, int(waves), int(slices), int(n_split), int(tp_block)))

    def tile_config(self) -> dict:
        out = (ctypes.c_int32 * 6)()
        _check(self._lib.xs_get_tile_config(self._h, out))
        return dict(waves=out[0], slices=out[1], n_split=out[2], tp_block=out[3], last_split=out[4],
                    last_block=out[5])

    def autotune(self, T: Sequence[float], P: Sequence[float], budget_ms: float = 2000.0) -> dict:
        T, P = list(T), list(P)
        if len(T) != len(P):
            raise ValueError("T and P differ in length")
        out = (ctypes.c_int32 * 4)()
        _check(self._lib.xs_autotune(self._h, len(T), _host_doubles(T), _host_doubles(P), float(budget_ms),
                                     self._stream(), out))
        return dict(waves=out[0], slices=out[1], n_split=out[2], tp_block=out[3])

    def graph(self, T: Sequence[float], P: Sequence[float], out=None) -> "Graph":
        """Capture the cross-section launch sequence for these (T, P) into `out`."""
        return Graph(self, T, P, out)

    def stream(self, T: Sequence[float], P: Sequence[float], out=None) -> "Stream":
        """Start accumulating cross sections over chunks of transitions from host memory."""
        return Stream(self, T, P, out)

    def set_timing(self, enable: bool = True):
        _check(self._lib.xs_set_timing(self._h, 1 if enable else 0))

    def kernel_times(self) -> dict:
        t = XsKernelTimes()
        _check(self._lib.xs_kernel_times(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in XsKernelTimes._fields_}

    def workspace_bytes(self) -> int:
        return int(self._lib.xs_workspace_bytes(self._h))


class Graph:
    """A captured xs_cross_section sequence; `sigma` is the output it writes on replay."""

    def __init__(self, plan: Plan, T: Sequence[float], P: Sequence[float], out=None):
        torch = plan._torch
        T, P = list(T), list(P)
        if len(T) != len(P):
            raise ValueError("T and P differ in length")
        if out is None:
            out = torch.empty((len(T), plan.n_points), dtype=plan.dtype, device="cuda")
        else:
            out = plan._dev(out, plan.dtype, "out")
            if out.numel() != len(T) * plan.n_points:
                raise ValueError("out has the wrong size")
        torch.cuda.synchronize()
        h = ctypes.c_void_p()
        _check(plan._lib.xs_graph_create(plan._h, len(T), _host_doubles(T), _host_doubles(P), _ptr(out),
                                         ctypes.byref(h)))
        self._plan = plan
        self._lib = plan._lib
        self._h = h
        self._pid = os.getpid()
        self.n_tp = len(T)
        self.sigma = out

    def set_tp(self, T: Sequence[float], P: Sequence[float]):
        T, P = list(T), list(P)
        if len(T) != self.n_tp or len(P) != self.n_tp:
            raise ValueError("T and P must keep the captured length")
        _check(self._lib.xs_graph_set_tp(self._h, _host_doubles(T), _host_doubles(P), self._plan._stream()))

    def launch(self):
        _check(self._lib.xs_graph_launch(self._h, self._plan._stream()))
        return self.sigma

    def workspace_bytes(self) -> int:
        return int(self._lib.xs_graph_workspace_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and _owner(self):
            self._lib.xs_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """Line-list streaming: chunks of transitions (host tensors, preferably pinned) are
    copied to the device while the previous chunk is computed; sums stay on the device."""

    def __init__(self, plan: Plan, T: Sequence[float] = (), P: Sequence[float] = (), out=None, *,
                 resume_from: Optional[str] = None, n_tp: Optional[int] = None):
        torch = plan._torch
        self._plan, self._lib = plan, plan._lib
        self._held = []
        h = ctypes.c_void_p()
        if resume_from is None:
            T, P = list(T), list(P)
            if len(T) != len(P):
                raise ValueError("T and P differ in length")
            n_tp = len(T)
        elif n_tp is None:
            raise ValueError("resuming needs n_tp (the checkpoint's number of (T, P) points)")
        if out is None:
            out = torch.empty((n_tp, plan.n_points), dtype=plan.dtype, device="cuda")
        else:
            out = plan._dev(out, plan.dtype, "out")
            if out.numel() != n_tp * plan.n_points:
                raise ValueError("out has the wrong size")
        if resume_from is None:
            _check(self._lib.xs_stream_begin(plan._h, n_tp, _host_doubles(T), _host_doubles(P), _ptr(out),
                                             plan._stream(), ctypes.byref(h)))
        else:
            _check(self._lib.xs_stream_resume(plan._h, os.fsencode(resume_from), _ptr(out), plan._stream(),
                                              ctypes.byref(h)))
        self._h = h
        self._pid = os.getpid()
        self.sigma = out

    @classmethod
    def resume(cls, plan: Plan, path: str, n_tp: int, out=None) -> "Stream":
        return cls(plan, out=out, resume_from=path, n_tp=n_tp)

    def _host(self, t, dtype, name):
        if t is None:
            return None
        if t.is_cuda or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous host tensor of {dtype}")
        return t

    def chunk(self, upper, lower, A, gamma_ref=None, n_exp=None):
        torch = self._plan._torch
        upper = self._host(upper, torch.int32, "upper")
        lower = self._host(lower, torch.int32, "lower")
        A = self._host(A, torch.float32, "A")
        gamma_ref = self._host(gamma_ref, torch.float32, "gamma_ref")
        n_exp = self._host(n_exp, torch.float32, "n_exp")
        n = _same_length("chunk", ("upper", upper), ("lower", lower), ("A", A), ("gamma_ref", gamma_ref),
                         ("n_exp", n_exp))
        self._plan._n_lines = None   # each chunk replaces the plan's line set
        _check(self._lib.xs_stream_chunk(self._h, n, _ptr(upper), _ptr(lower), _ptr(A),
                                         _ptr(gamma_ref), _ptr(n_exp)))
        # the host arrays must outlive their asynchronous copy (until the next call returns)
        self._held = [upper, lower, A, gamma_ref, n_exp]

    def chunk_device(self, upper, lower, A, gamma_ref=None, n_exp=None):
        """A chunk whose arrays already live on the GPU (no copy; computed during the call)."""
        plan = self._plan
        torch = plan._torch
        upper = plan._dev(upper, torch.int32, "upper")
        lower = plan._dev(lower, torch.int32, "lower")
        A = plan._dev(A, torch.float32, "A")
        gamma_ref = plan._dev(gamma_ref, torch.float32, "gamma_ref")
        n_exp = plan._dev(n_exp, torch.float32, "n_exp")
        n = _same_length("chunk_device", ("upper", upper), ("lower", lower), ("A", A), ("gamma_ref", gamma_ref),
                         ("n_exp", n_exp))
        plan._n_lines = None   # each chunk replaces the plan's line set
        _check(self._lib.xs_stream_chunk_device(self._h, n, _ptr(upper), _ptr(lower), _ptr(A), _ptr(gamma_ref),
                                                _ptr(n_exp)))

    def checkpoint(self, path: str):
        _check(self._lib.xs_stream_checkpoint(self._h, os.fsencode(path)))

    def stats(self) -> dict:
        out = (ctypes.c_int64 * 3)()
        _check(self._lib.xs_stream_stats(self._h, out))
        return dict(chunks=out[0], lines=out[1], kept=out[2])

    def end(self):
        """Finish: returns (sigma, lines kept); the stream is released."""
        kept = ctypes.c_int64()
        h, self._h = self._h, ctypes.c_void_p()
        _check(self._lib.xs_stream_end(h, ctypes.byref(kept)))
        self._held = []
        return self.sigma, int(kept.value)

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None and self._h.value and _owner(self):
                self._lib.xs_stream_end(self._h, None)
        except Exception:
            pass
