"""ctypes binding of libconv.so (include/conv.h).

Argument marshalling only: torch tensors supply device memory and the stream; every step of the
scheme runs in the library's HIP kernels.  There is no CPU path: if the library is missing or no
GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libconv.so")

CONV_OK, CONV_EINVAL, CONV_EUNSUPPORTED, CONV_EHIP, CONV_ERANGE = 0, -1, -2, -3, -4

PARAM_FIELDS = (
    "cape_threshold", "tau", "eps_deep", "alpha_dd", "evap_max_frac", "p_launch_min", "p_top_min",
    "eps_sh", "delta_sh", "qlcrit_sh", "cin_max", "a_buoy", "b_drag", "c_tke", "p_lcl_min",
    "p_sh_top_min", "eps_cape",
)
DEFAULTS = dict(
    cape_threshold=70.0, tau=3600.0, eps_deep=1.0e-4, alpha_dd=0.2, evap_max_frac=0.9,
    p_launch_min=60000.0, p_top_min=4000.0, eps_sh=1.0e-3, delta_sh=1.0e-3, qlcrit_sh=1.0e-3,
    cin_max=100.0, a_buoy=1.0, b_drag=1.0, c_tke=1.0, p_lcl_min=60000.0, p_sh_top_min=40000.0,
    eps_cape=0.0,
)

EXPORTS = ("conv_workspace_bytes", "conv_create", "conv_set_params", "conv_destroy",
           "conv_deep_forward", "conv_shallow_forward", "conv_step", "conv_set_launch",
           "conv_get_launch", "conv_step_static", "conv_timing_start",
           "conv_timing_read", "conv_strerror", "conv_last_hip_error",
           "conv_backward_workspace_bytes", "conv_deep_backward", "conv_shallow_backward",
           "conv_step_backward", "conv_tracer_transport", "conv_momentum_transport",
           "conv_autotune",
           "conv_ensemble_workspace_bytes", "conv_ensemble_create", "conv_ensemble_destroy",
           "conv_ensemble_step", "conv_ensemble_set_launch", "conv_ensemble_get_launch",
           "conv_ensemble_autotune", "conv_ensemble_capture", "conv_ensemble_replay",
           "mlp_workspace_bytes", "mlp_create", "mlp_workspace_bytes_ex", "mlp_create_ex",
           "mlp_destroy", "mlp_param_count", "mlp_set_params",
           "mlp_get_params", "mlp_get_grads", "mlp_forward", "mlp_mse", "mlp_backward",
           "mlp_adam_step", "mlp_train_step", "mlp_gemm_nt", "mlp_strerror",
           "surr_pack_inputs_raw", "surr_pack_targets_raw", "surr_col_stats_scratch_bytes",
           "surr_col_stats", "surr_normalize", "surr_pack_inputs", "surr_workspace_bytes",
           "surr_create", "surr_destroy", "surr_set_norm", "surr_set_fused", "surr_infer")


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in PARAM_FIELDS]


class State(C.Structure):
    _fields_ = [("T", C.c_void_p), ("q", C.c_void_p), ("p_mid", C.c_void_p), ("z", C.c_void_p),
                ("p_int", C.c_void_p), ("phis", C.c_void_p), ("pblh", C.c_void_p),
                ("tke", C.c_void_p), ("ld", C.c_int64), ("dt", C.c_double)]


class DeepOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("dTdt", "dqdt", "mu", "md", "prec", "cape", "klaunch",
                                          "ktop", "trig", "status")]


class ShallowOut(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("dTdt", "dqdt", "mu", "prec", "cin", "kbase", "ktop",
                                          "status")]


class DeepCot(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("g_dTdt", "g_dqdt", "g_prec")]


class DeepGrad(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("g_T", "g_q", "g_params")]


ShallowCot = DeepCot    # {g_dTdt, g_dqdt, g_prec}: the same three device pointers
ShallowGrad = DeepGrad  # {g_T, g_q, g_params}; g_params has 2 entries (eps_sh, delta_sh)
StepGrad = DeepGrad     # {g_T, g_q, g_params}; g_params has 4 entries


class Member(C.Structure):
    _fields_ = [("ncol", C.c_int64), ("nlev", C.c_int32), ("params", Params), ("state", State),
                ("deep", DeepOut), ("shallow", ShallowOut)]


_lib = None


def lib():
    """Load libconv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1711_00289_amd.build` (there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        L.conv_workspace_bytes.restype = C.c_size_t
        L.conv_workspace_bytes.argtypes = [C.c_int64, C.c_int32]
        L.conv_create.restype = C.c_int
        L.conv_create.argtypes = [C.c_int64, C.c_int32, C.POINTER(Params), C.c_void_p, C.c_size_t,
                                  C.POINTER(C.c_void_p)]
        L.conv_set_params.restype = C.c_int
        L.conv_set_params.argtypes = [C.c_void_p, C.POINTER(Params)]
        L.conv_destroy.restype = None
        L.conv_destroy.argtypes = [C.c_void_p]
        L.conv_deep_forward.restype = C.c_int
        L.conv_deep_forward.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(DeepOut), C.c_void_p]
        L.conv_shallow_forward.restype = C.c_int
        L.conv_shallow_forward.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(ShallowOut),
                                           C.c_void_p]
        L.conv_step.restype = C.c_int
        L.conv_step.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(DeepOut),
                                C.POINTER(ShallowOut), C.c_void_p]
        L.conv_step_static.restype = C.c_int
        L.conv_step_static.argtypes = [C.c_int64, C.c_int32, C.POINTER(Params), C.POINTER(State),
                                       C.POINTER(DeepOut), C.POINTER(ShallowOut), C.c_void_p]
        L.conv_set_launch.restype = C.c_int
        L.conv_set_launch.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.conv_get_launch.restype = C.c_int
        L.conv_get_launch.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.conv_timing_start.restype = C.c_int
        L.conv_timing_start.argtypes = [C.c_void_p, C.c_int]
        L.conv_timing_read.restype = C.c_int
        L.conv_timing_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.conv_backward_workspace_bytes.restype = C.c_size_t
        L.conv_backward_workspace_bytes.argtypes = [C.c_int64, C.c_int32, C.c_int64]
        L.conv_shallow_backward.restype = C.c_int
        L.conv_shallow_backward.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(ShallowOut),
                                            C.POINTER(ShallowCot), C.POINTER(ShallowGrad),
                                            C.c_void_p, C.c_size_t, C.c_void_p]
        L.conv_step_backward.restype = C.c_int
        L.conv_step_backward.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(DeepOut),
                                         C.POINTER(ShallowOut), C.POINTER(DeepCot),
                                         C.POINTER(ShallowCot), C.POINTER(StepGrad), C.c_void_p,
                                         C.c_size_t, C.c_void_p]
        L.conv_tracer_transport.restype = C.c_int
        L.conv_tracer_transport.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(DeepOut),
                                            C.POINTER(ShallowOut), C.c_int32, C.c_void_p,
                                            C.c_void_p, C.c_void_p, C.c_void_p]
        L.conv_momentum_transport.restype = C.c_int
        L.conv_momentum_transport.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(DeepOut),
                                              C.POINTER(ShallowOut), C.c_void_p, C.c_double,
                                              C.c_void_p, C.c_void_p, C.c_void_p]
        L.conv_deep_backward.restype = C.c_int
        L.conv_deep_backward.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(DeepOut),
                                         C.POINTER(DeepCot), C.POINTER(DeepGrad), C.c_void_p,
                                         C.c_size_t, C.c_void_p]
        I, P = C.c_int, C.POINTER(C.c_int)
        L.conv_autotune.restype = I
        L.conv_autotune.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(DeepOut),
                                    C.POINTER(ShallowOut), C.c_void_p, I, I, P, P,
                                    C.POINTER(C.c_float)]
        L.conv_ensemble_workspace_bytes.restype = C.c_size_t
        L.conv_ensemble_workspace_bytes.argtypes = [I, C.POINTER(Member)]
        L.conv_ensemble_create.restype = I
        L.conv_ensemble_create.argtypes = [I, C.POINTER(Member), C.c_void_p, C.c_size_t,
                                           C.POINTER(C.c_void_p)]
        L.conv_ensemble_destroy.restype = None
        L.conv_ensemble_destroy.argtypes = [C.c_void_p]
        for f in ("conv_ensemble_step", "conv_ensemble_capture", "conv_ensemble_replay"):
            getattr(L, f).restype = I
            getattr(L, f).argtypes = [C.c_void_p, C.c_void_p]
        L.conv_ensemble_set_launch.restype = I
        L.conv_ensemble_set_launch.argtypes = [C.c_void_p, I, I]
        L.conv_ensemble_get_launch.restype = I
        L.conv_ensemble_get_launch.argtypes = [C.c_void_p, P, P]
        L.conv_ensemble_autotune.restype = I
        L.conv_ensemble_autotune.argtypes = [C.c_void_p, C.c_void_p, I, I, P, P,
                                             C.POINTER(C.c_float)]
        V, I64 = C.c_void_p, C.c_int64
        L.mlp_workspace_bytes.restype = C.c_size_t
        L.mlp_workspace_bytes.argtypes = [C.POINTER(C.c_int32), I, I64]
        L.mlp_create.restype = I
        L.mlp_create.argtypes = [C.POINTER(C.c_int32), I, I64, V, C.c_size_t, C.POINTER(V)]
        L.mlp_workspace_bytes_ex.restype = C.c_size_t
        L.mlp_workspace_bytes_ex.argtypes = [C.POINTER(C.c_int32), I, I64, I64]
        L.mlp_create_ex.restype = I
        L.mlp_create_ex.argtypes = [C.POINTER(C.c_int32), I, I64, I64, V, C.c_size_t,
                                    C.POINTER(V)]
        L.mlp_destroy.restype = None
        L.mlp_destroy.argtypes = [V]
        L.mlp_param_count.restype = I64
        L.mlp_param_count.argtypes = [V]
        for f in ("mlp_set_params", "mlp_get_params", "mlp_get_grads"):
            getattr(L, f).restype = I
            getattr(L, f).argtypes = [V, V, V]
        L.mlp_forward.restype = I
        L.mlp_forward.argtypes = [V, V, V, I64, I, V]
        L.mlp_mse.restype = I
        L.mlp_mse.argtypes = [V, V, V, I64, I, V, V]
        L.mlp_backward.restype = I
        L.mlp_backward.argtypes = [V, I64, V]
        L.mlp_adam_step.restype = I
        L.mlp_adam_step.argtypes = [V, C.c_float, C.c_float, C.c_float, C.c_float, V]
        L.mlp_train_step.restype = I
        L.mlp_train_step.argtypes = [V, V, V, I64, I, C.c_float, C.c_float, C.c_float, C.c_float,
                                     V, V, V]
        L.mlp_gemm_nt.restype = I
        L.mlp_gemm_nt.argtypes = [V, I64, V, I64, V, I64, C.c_int32, C.c_int32, I, V, I64, V, V]
        L.mlp_strerror.restype = C.c_char_p
        L.mlp_strerror.argtypes = [I]
        L.surr_pack_inputs_raw.restype = I
        L.surr_pack_inputs_raw.argtypes = [C.POINTER(State), C.c_int32, I64, C.c_int32, V, V]
        L.surr_pack_targets_raw.restype = I
        L.surr_pack_targets_raw.argtypes = [C.POINTER(DeepOut), C.POINTER(ShallowOut), C.c_int32, I64,
                                            I64, C.c_int32, V, V]
        L.surr_col_stats_scratch_bytes.restype = C.c_size_t
        L.surr_col_stats_scratch_bytes.argtypes = [C.c_int32]
        L.surr_col_stats.restype = I
        L.surr_col_stats.argtypes = [V, I64, C.c_int32, C.c_int32, V, V, V, V, C.c_size_t, V]
        L.surr_normalize.restype = I
        L.surr_normalize.argtypes = [V, I64, C.c_int32, V, V, V, V]
        L.surr_pack_inputs.restype = I
        L.surr_pack_inputs.argtypes = [C.POINTER(State), C.c_int32, I64, C.c_int32, V, V, V, V]
        L.surr_workspace_bytes.restype = C.c_size_t
        L.surr_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, I64, I64]
        L.surr_create.restype = I
        L.surr_create.argtypes = [V, C.c_int32, C.c_int32, C.c_int32, I64, I64, C.POINTER(Params), V,
                                  C.c_size_t, C.POINTER(V)]
        L.surr_destroy.restype = None
        L.surr_destroy.argtypes = [V]
        L.surr_set_norm.restype = I
        L.surr_set_norm.argtypes = [V, V, V, V, V, C.c_double, C.c_double, V]
        L.surr_set_fused.restype = I
        L.surr_set_fused.argtypes = [V, I]
        L.surr_infer.restype = I
        L.surr_infer.argtypes = [V, C.POINTER(State), I64, V, V, V, I, C.POINTER(I64), V]
        L.conv_strerror.restype = C.c_char_p
        L.conv_strerror.argtypes = [C.c_int]
        L.conv_last_hip_error.restype = C.c_int
        L.conv_last_hip_error.argtypes = []
        _lib = L
    return _lib


def make_params(**over) -> Params:
    d = dict(DEFAULTS)
    for k, v in over.items():
        if k not in d:
            raise KeyError(k)
        d[k] = float(v)
    return Params(*[d[n] for n in PARAM_FIELDS])


def check(rc: int, what: str):
    if rc != CONV_OK:
        msg = lib().conv_strerror(rc).decode()
        if rc == CONV_EHIP:
            msg += f" (hipError {lib().conv_last_hip_error()})"
        raise RuntimeError(f"{what}: {msg}")


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("libconv needs a ROCm GPU (torch.cuda is not available)")
    return torch


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_device(st: dict, device="cuda"):
    """Copy a level-major numpy state dict (from soundings.make_state) to device tensors (the
    arrays' width is the state's leading dimension)."""
    torch = _torch()
    out = {}
    for k in ("T", "q", "p_mid", "z", "p_int", "phis", "pblh", "tke"):
        out[k] = torch.as_tensor(st[k], dtype=torch.float64).to(device).contiguous()
    out["dt"] = float(st["dt"])
    out["ncol"] = int(st.get("ncol", st["T"].shape[1]))
    return out


def alloc_deep(torch, device, nlev: int, ld: int) -> dict:
    """Device output arrays of the deep scheme for `ld` columns."""
    f = lambda *sh: torch.empty(*sh, dtype=torch.float64, device=device)
    i = lambda n: torch.empty(n, dtype=torch.int32, device=device)
    L = nlev
    return dict(dTdt=f(L, ld), dqdt=f(L, ld), mu=f(L + 1, ld), md=f(L + 1, ld), prec=f(ld),
                cape=f(ld), klaunch=i(ld), ktop=i(ld), trig=i(ld), status=i(ld))


def alloc_shallow(torch, device, nlev: int, ld: int) -> dict:
    """Device output arrays of the shallow scheme for `ld` columns."""
    f = lambda *sh: torch.empty(*sh, dtype=torch.float64, device=device)
    i = lambda n: torch.empty(n, dtype=torch.int32, device=device)
    L = nlev
    return dict(dTdt=f(L, ld), dqdt=f(L, ld), mu=f(L + 1, ld), prec=f(ld), cin=f(ld),
                kbase=i(ld), ktop=i(ld), status=i(ld))


def state_struct(torch, s: dict, nlev: int, ncol: int) -> State:
    """conv_state_t over a device state dict, after checking shapes, dtypes and contiguity."""
    T = s["T"]
    if T.dim() != 2 or T.shape[0] != nlev or T.shape[1] < ncol:
        raise ValueError("state arrays must be [nlev][ld] with ld >= ncol")
    ld = T.shape[1]
    for k, rows in (("T", nlev), ("q", nlev), ("p_mid", nlev), ("z", nlev), ("p_int", nlev + 1)):
        a = s[k]
        if a.dtype != torch.float64 or not a.is_contiguous() or tuple(a.shape) != (rows, ld):
            raise ValueError(f"{k}: expected contiguous float64 [{rows}][{ld}]")
    for k in ("phis", "pblh", "tke"):
        a = s[k]
        if a.dtype != torch.float64 or a.numel() < ld:
            raise ValueError(f"{k}: expected float64 [{ld}]")
    return State(*[s[k].data_ptr() for k in ("T", "q", "p_mid", "z", "p_int", "phis", "pblh",
                                              "tke")], ld, float(s["dt"]))


def step_static(s: dict, ncol: int, nlev: int, deep: dict, shallow: dict,
                params: Params | None = None, stream=None) -> int:
    """conv_step_static: one step over columns 0..ncol-1 of the device state `s` into the
    preallocated device outputs `deep` and `shallow`, with the library's static device scratch as
    the workspace (nothing is allocated).  Returns the library's code (CONV_OK, or CONV_ERANGE for
    sizes beyond the static scratch); raises on other errors."""
    torch = _torch()
    st = state_struct(torch, s, nlev, ncol)
    params = params or make_params()
    d = DeepOut(*[deep[f].data_ptr() for f, _ in DeepOut._fields_])
    h = ShallowOut(*[shallow[f].data_ptr() for f, _ in ShallowOut._fields_])
    strm = C.c_void_p(stream.cuda_stream) if stream is not None else _stream(torch)
    rc = lib().conv_step_static(int(ncol), int(nlev), C.byref(params), C.byref(st), C.byref(d),
                                C.byref(h), strm)
    if rc != CONV_ERANGE:
        check(rc, "conv_step_static")
    return rc


class Conv:
    """A context over `ncol` columns of `nlev` levels with a torch-allocated workspace."""

    def __init__(self, ncol: int, nlev: int, params: Params | None = None, device="cuda"):
        torch = _torch()
        self.torch = torch
        self.ncol, self.nlev = int(ncol), int(nlev)
        self.device = device
        L = lib()
        nbytes = L.conv_workspace_bytes(self.ncol, self.nlev)
        if nbytes == 0:
            raise ValueError("unsupported size")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.params = params or make_params()
        h = C.c_void_p()
        check(L.conv_create(self.ncol, self.nlev, C.byref(self.params), C.c_void_p(self.ws_ptr),
                            nbytes, C.byref(h)), "conv_create")
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().conv_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_params(self, params: Params):
        self.params = params
        check(lib().conv_set_params(self.h, C.byref(params)), "conv_set_params")

    # -- outputs -------------------------------------------------------------------------
    def _f64(self, *shape):
        return self.torch.empty(*shape, dtype=self.torch.float64, device=self.device)

    def alloc_deep(self, ld: int):
        return alloc_deep(self.torch, self.device, self.nlev, ld)

    def alloc_shallow(self, ld: int):
        return alloc_shallow(self.torch, self.device, self.nlev, ld)

    # -- marshalling ---------------------------------------------------------------------
    def _state(self, s: dict) -> State:
        return state_struct(self.torch, s, self.nlev, self.ncol)

    @staticmethod
    def _deep_struct(o):
        return DeepOut(*[o[f].data_ptr() for f, _ in DeepOut._fields_])

    @staticmethod
    def _shallow_struct(o):
        return ShallowOut(*[o[f].data_ptr() for f, _ in ShallowOut._fields_])

    # -- calls ---------------------------------------------------------------------------
    def deep_forward(self, s: dict, out: dict | None = None) -> dict:
        st = self._state(s)
        out = out or self.alloc_deep(st.ld)
        o = self._deep_struct(out)
        check(lib().conv_deep_forward(self.h, C.byref(st), C.byref(o), _stream(self.torch)),
              "conv_deep_forward")
        return out

    def shallow_forward(self, s: dict, out: dict | None = None) -> dict:
        st = self._state(s)
        out = out or self.alloc_shallow(st.ld)
        o = self._shallow_struct(out)
        check(lib().conv_shallow_forward(self.h, C.byref(st), C.byref(o), _stream(self.torch)),
              "conv_shallow_forward")
        return out

    def step(self, s: dict, deep: dict | None = None, shallow: dict | None = None):
        st = self._state(s)
        deep = deep or self.alloc_deep(st.ld)
        shallow = shallow or self.alloc_shallow(st.ld)
        d, h = self._deep_struct(deep), self._shallow_struct(shallow)
        check(lib().conv_step(self.h, C.byref(st), C.byref(d), C.byref(h), _stream(self.torch)),
              "conv_step")
        return deep, shallow

    def _cotangents(self, ld, g_dTdt, g_dqdt, g_prec):
        torch = self.torch

        def cot(a, shape):
            if a is None:
                return None
            if a.dtype != torch.float64 or tuple(a.shape) != shape:
                raise ValueError(f"cotangent: expected float64 {shape}")
            return a.contiguous()

        return (cot(g_dTdt, (self.nlev, ld)), cot(g_dqdt, (self.nlev, ld)), cot(g_prec, (ld,)))

    @staticmethod
    def _cot_struct(cs):
        return DeepCot(*[a.data_ptr() if a is not None else None for a in cs])

    def _backward_workspace(self, ld):
        nbytes = lib().conv_backward_workspace_bytes(self.ncol, self.nlev, ld)
        if nbytes == 0:
            raise ValueError("unsupported size")
        if getattr(self, "_bws", None) is None or self._bws.numel() < nbytes + 256:
            self._bws = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        return C.c_void_p((self._bws.data_ptr() + 255) & ~255), nbytes

    def deep_backward(self, s: dict, fwd: dict, g_dTdt=None, g_dqdt=None, g_prec=None):
        """Adjoint of deep_forward at state `s` (with `fwd` its outputs): returns dict(g_T, g_q,
        g_tau, g_eps) for the cotangents given (None = zero)."""
        st = self._state(s)
        ld = st.ld
        cs = self._cotangents(ld, g_dTdt, g_dqdt, g_prec)
        wptr, nbytes = self._backward_workspace(ld)
        gT, gq, gp = self._f64(self.nlev, ld), self._f64(self.nlev, ld), self._f64(2)
        c = self._cot_struct(cs)
        g = DeepGrad(gT.data_ptr(), gq.data_ptr(), gp.data_ptr())
        o = self._deep_struct(fwd)
        check(lib().conv_deep_backward(self.h, C.byref(st), C.byref(o), C.byref(c), C.byref(g),
                                       wptr, nbytes, _stream(self.torch)), "conv_deep_backward")
        return dict(g_T=gT, g_q=gq, g_tau=gp[0], g_eps=gp[1])

    def shallow_backward(self, s: dict, fwd: dict, g_dTdt=None, g_dqdt=None, g_prec=None):
        """Adjoint of shallow_forward at state `s` (with `fwd` its outputs): returns dict(g_T,
        g_q, g_eps_sh, g_delta_sh) for the cotangents given (None = zero)."""
        st = self._state(s)
        ld = st.ld
        cs = self._cotangents(ld, g_dTdt, g_dqdt, g_prec)
        wptr, nbytes = self._backward_workspace(ld)
        gT, gq, gp = self._f64(self.nlev, ld), self._f64(self.nlev, ld), self._f64(2)
        c = self._cot_struct(cs)
        g = ShallowGrad(gT.data_ptr(), gq.data_ptr(), gp.data_ptr())
        o = self._shallow_struct(fwd)
        check(lib().conv_shallow_backward(self.h, C.byref(st), C.byref(o), C.byref(c), C.byref(g),
                                          wptr, nbytes, _stream(self.torch)),
              "conv_shallow_backward")
        return dict(g_T=gT, g_q=gq, g_eps_sh=gp[0], g_delta_sh=gp[1])

    def step_backward(self, s: dict, deep: dict, shallow: dict, deep_cot=(None, None, None),
                      shallow_cot=(None, None, None)):
        """Adjoint of step at state `s` (with `deep`, `shallow` its outputs), for cotangents
        (g_dTdt, g_dqdt, g_prec) of each scheme's outputs (None = zero): returns dict(g_T, g_q,
        g_tau, g_eps, g_eps_sh, g_delta_sh)."""
        st = self._state(s)
        ld = st.ld
        dc = self._cot_struct(self._cotangents(ld, *deep_cot))
        sc = self._cot_struct(self._cotangents(ld, *shallow_cot))
        wptr, nbytes = self._backward_workspace(ld)
        gT, gq, gp = self._f64(self.nlev, ld), self._f64(self.nlev, ld), self._f64(4)
        g = StepGrad(gT.data_ptr(), gq.data_ptr(), gp.data_ptr())
        d, h = self._deep_struct(deep), self._shallow_struct(shallow)
        check(lib().conv_step_backward(self.h, C.byref(st), C.byref(d), C.byref(h), C.byref(dc),
                                       C.byref(sc), C.byref(g), wptr, nbytes, _stream(self.torch)),
              "conv_step_backward")
        return dict(g_T=gT, g_q=gq, g_tau=gp[0], g_eps=gp[1], g_eps_sh=gp[2], g_delta_sh=gp[3])

    def tracer_transport(self, s: dict, deep: dict, shallow: dict, tracers, deep_part=False,
                         out=None):
        """Convective transport of tracers [ntr][nlev][ld] (float64, device) by the plumes of the
        step whose outputs are `deep`, `shallow`: returns the deep + shallow tendency, and with
        deep_part also the deep part alone."""
        torch = self.torch
        st = self._state(s)
        if tracers.dtype != torch.float64 or tracers.dim() != 3 or tuple(tracers.shape[1:]) != (
                self.nlev, st.ld):
            raise ValueError(f"tracers: expected float64 [ntr][{self.nlev}][{st.ld}]")
        tr = tracers.contiguous()
        tend = out if out is not None else torch.empty_like(tr)
        dpart = torch.empty_like(tr) if deep_part else None
        d, h = self._deep_struct(deep), self._shallow_struct(shallow)
        check(lib().conv_tracer_transport(self.h, C.byref(st), C.byref(d), C.byref(h),
                                          int(tr.shape[0]), tr.data_ptr(), tend.data_ptr(),
                                          dpart.data_ptr() if dpart is not None else None,
                                          _stream(torch)), "conv_tracer_transport")
        return (tend, dpart) if deep_part else tend

    def momentum_transport(self, s: dict, deep: dict, shallow: dict, wind, c_pgf: float = 0.7,
                           deep_part=False, out=None):
        """Convective momentum transport of wind [2][nlev][ld] (u, v; float64, device) by the
        plumes of the step whose outputs are `deep`, `shallow`, with pressure-gradient coefficient
        c_pgf: returns the deep + shallow tendency, and with deep_part also the deep part alone."""
        torch = self.torch
        st = self._state(s)
        if wind.dtype != torch.float64 or tuple(wind.shape) != (2, self.nlev, st.ld):
            raise ValueError(f"wind: expected float64 [2][{self.nlev}][{st.ld}]")
        w = wind.contiguous()
        tend = out if out is not None else torch.empty_like(w)
        dpart = torch.empty_like(w) if deep_part else None
        d, h = self._deep_struct(deep), self._shallow_struct(shallow)
        check(lib().conv_momentum_transport(self.h, C.byref(st), C.byref(d), C.byref(h),
                                            w.data_ptr(), float(c_pgf), tend.data_ptr(),
                                            dpart.data_ptr() if dpart is not None else None,
                                            _stream(torch)), "conv_momentum_transport")
        return (tend, dpart) if deep_part else tend

    def autotune(self, s: dict, deep: dict, shallow: dict, reps: int = 5, force: bool = False):
        """Pick the fastest persistent-grid shape for conv_step on these arrays (cached per
        process); returns (fused_waves_per_cu, shallow_waves_per_cu, median_ms)."""
        st = self._state(s)
        d, h = self._deep_struct(deep), self._shallow_struct(shallow)
        a, b, ms = C.c_int(0), C.c_int(0), C.c_float(0.0)
        check(lib().conv_autotune(self.h, C.byref(st), C.byref(d), C.byref(h), _stream(self.torch),
                                  int(reps), int(force), C.byref(a), C.byref(b), C.byref(ms)),
              "conv_autotune")
        return a.value, b.value, ms.value

    # -- instrumentation -----------------------------------------------------------------
    STAGES = ("reset", "trigger", "deep_plume", "shallow_retrigger", "shallow_plume")

    def set_launch(self, fused_waves_per_cu: int, shallow_waves_per_cu: int):
        check(lib().conv_set_launch(self.h, int(fused_waves_per_cu), int(shallow_waves_per_cu)),
              "conv_set_launch")

    def get_launch(self):
        a, b = C.c_int(0), C.c_int(0)
        check(lib().conv_get_launch(self.h, C.byref(a), C.byref(b)), "conv_get_launch")
        return a.value, b.value

    def timing_start(self, max_calls: int):
        check(lib().conv_timing_start(self.h, int(max_calls)), "conv_timing_start")

    def timing_read(self):
        ms = (C.c_double * len(self.STAGES))()
        n = C.c_int(0)
        check(lib().conv_timing_read(self.h, ms, C.byref(n)), "conv_timing_read")
        return {s: ms[i] for i, s in enumerate(self.STAGES)}, n.value


def _autograd():
    import torch

    class DeepConv(torch.autograd.Function):
        """(T, q, tau, eps_deep) -> (dTdt, dqdt, prec) of the deep scheme, differentiable through
        the library's hand-written adjoint (branches of the forward run held fixed)."""

        @staticmethod
        def forward(ctx, T, q, tau, eps_deep, conv, state):
            import copy

            p = copy.copy(conv.params)
            p.tau = float(tau)
            p.eps_deep = float(eps_deep)
            conv.set_params(p)
            s = dict(state)
            s["T"], s["q"] = T.detach().contiguous(), q.detach().contiguous()
            out = conv.deep_forward(s)
            ctx.conv, ctx.s, ctx.out = conv, s, out
            ctx.params = p
            ctx.shapes = (tau.shape, eps_deep.shape)
            return out["dTdt"].clone(), out["dqdt"].clone(), out["prec"].clone()

        @staticmethod
        def backward(ctx, gT, gq, gP):
            conv = ctx.conv
            conv.set_params(ctx.params)
            g = conv.deep_backward(ctx.s, ctx.out, gT, gq, gP)
            return (g["g_T"], g["g_q"], g["g_tau"].reshape(ctx.shapes[0]),
                    g["g_eps"].reshape(ctx.shapes[1]), None, None)

    class StepConv(torch.autograd.Function):
        """(T, q, p) -> the deep and shallow (dTdt, dqdt, prec) of one step, p = (tau, eps_deep,
        eps_sh, delta_sh) as a 4-vector, differentiable through conv_step_backward."""

        @staticmethod
        def forward(ctx, T, q, p4, conv, state):
            import copy

            p = copy.copy(conv.params)
            p.tau, p.eps_deep, p.eps_sh, p.delta_sh = (float(v) for v in p4.detach().cpu())
            conv.set_params(p)
            s = dict(state)
            s["T"], s["q"] = T.detach().contiguous(), q.detach().contiguous()
            deep, shallow = conv.step(s)
            ctx.conv, ctx.s, ctx.deep, ctx.shallow, ctx.params = conv, s, deep, shallow, p
            ctx.pshape, ctx.pdevice = p4.shape, p4.device
            return tuple(o[k].clone() for o in (deep, shallow) for k in ("dTdt", "dqdt", "prec"))

        @staticmethod
        def backward(ctx, gdT, gdq, gdP, gsT, gsq, gsP):
            conv = ctx.conv
            conv.set_params(ctx.params)
            g = conv.step_backward(ctx.s, ctx.deep, ctx.shallow, (gdT, gdq, gdP), (gsT, gsq, gsP))
            gp = torch.stack([g["g_tau"], g["g_eps"], g["g_eps_sh"], g["g_delta_sh"]])
            return g["g_T"], g["g_q"], gp.reshape(ctx.pshape).to(ctx.pdevice), None, None

    return DeepConv, StepConv


_DeepConv = None
_StepConv = None


def deep_conv(conv: "Conv", state: dict, T, q, tau, eps_deep):
    """Differentiable deep convection: returns (dTdt, dqdt, prec); gradients flow to T, q and the
    0-d tensors tau, eps_deep through conv_deep_backward."""
    global _DeepConv, _StepConv
    if _DeepConv is None:
        _DeepConv, _StepConv = _autograd()
    return _DeepConv.apply(T, q, tau, eps_deep, conv, state)


def step_conv(conv: "Conv", state: dict, T, q, p4):
    """Differentiable step (deep, state update, shallow): returns the deep (dTdt, dqdt, prec) and
    the shallow (dTdt, dqdt, prec); gradients flow to T, q and the 4-vector p4 = (tau, eps_deep,
    eps_sh, delta_sh) through conv_step_backward."""
    global _DeepConv, _StepConv
    if _StepConv is None:
        _DeepConv, _StepConv = _autograd()
    return _StepConv.apply(T, q, p4, conv, state)


class Ensemble:
    """Several grids stepped by the same launches (conv_ensemble_*).  `members` is a list of dicts
    with a device state (from to_device), `nlev`, and optionally `params`, `deep`, `shallow`
    (output dicts as from Conv.alloc_*; allocated here when missing)."""

    def __init__(self, members, device="cuda"):
        torch = _torch()
        self.torch = torch
        self.device = device
        self.members = []
        tab = (Member * len(members))()
        for i, m in enumerate(members):
            s = m["state"]
            nlev = int(m["nlev"])
            ncol = int(m.get("ncol", s["ncol"]))
            ld = s["T"].shape[1]
            deep = m.get("deep") or alloc_deep(torch, device, nlev, ld)
            shallow = m.get("shallow") or alloc_shallow(torch, device, nlev, ld)
            params = m.get("params") or make_params()
            tab[i] = Member(ncol, nlev, params, state_struct(torch, s, nlev, ncol),
                            Conv._deep_struct(deep), Conv._shallow_struct(shallow))
            self.members.append(dict(state=s, nlev=nlev, ncol=ncol, params=params, deep=deep,
                                     shallow=shallow))
        self.tab = tab
        L = lib()
        nbytes = L.conv_ensemble_workspace_bytes(len(members), tab)
        if nbytes == 0:
            raise ValueError("malformed ensemble members")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        wptr = (self.ws.data_ptr() + 255) & ~255
        h = C.c_void_p()
        check(L.conv_ensemble_create(len(members), tab, C.c_void_p(wptr), nbytes, C.byref(h)),
              "conv_ensemble_create")
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().conv_ensemble_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def step(self, stream=None):
        check(lib().conv_ensemble_step(self.h, self._s(stream)), "conv_ensemble_step")

    def _s(self, stream):
        if stream is None:
            return _stream(self.torch)
        return C.c_void_p(stream.cuda_stream)

    def set_launch(self, fused: int, shallow: int):
        check(lib().conv_ensemble_set_launch(self.h, int(fused), int(shallow)),
              "conv_ensemble_set_launch")

    def get_launch(self):
        a, b = C.c_int(0), C.c_int(0)
        check(lib().conv_ensemble_get_launch(self.h, C.byref(a), C.byref(b)),
              "conv_ensemble_get_launch")
        return a.value, b.value

    def autotune(self, reps: int = 5, force: bool = False, stream=None):
        a, b, ms = C.c_int(0), C.c_int(0), C.c_float(0.0)
        check(lib().conv_ensemble_autotune(self.h, self._s(stream), int(reps), int(force),
                                           C.byref(a), C.byref(b), C.byref(ms)),
              "conv_ensemble_autotune")
        return a.value, b.value, ms.value

    def capture(self, stream):
        """Capture one step into a HIP graph on `stream` (a torch.cuda.Stream, not the default)."""
        check(lib().conv_ensemble_capture(self.h, C.c_void_p(stream.cuda_stream)),
              "conv_ensemble_capture")

    def replay(self, stream):
        check(lib().conv_ensemble_replay(self.h, C.c_void_p(stream.cuda_stream)),
              "conv_ensemble_replay")


def mlp_check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what}: {lib().mlp_strerror(rc).decode()}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class MLP:
    """The surrogate network (include/mlp.h) over a torch-allocated workspace.  Inputs are
    torch.bfloat16 [batch][widths[0]]; outputs and targets float32 [batch][widths[-1]].
    `max_train_batch` (default max_batch) bounds the training forwards and backwards only."""

    def __init__(self, widths, max_batch: int, device="cuda", max_train_batch: int | None = None):
        torch = _torch()
        self.torch = torch
        self.widths = [int(w) for w in widths]
        self.n = len(self.widths) - 1
        self.max_batch = int(max_batch)
        self.max_train_batch = int(max_train_batch or max_batch)
        self.device = device
        warr = (C.c_int32 * len(self.widths))(*self.widths)
        self._warr = warr
        L = lib()
        nbytes = L.mlp_workspace_bytes_ex(warr, self.n, self.max_batch, self.max_train_batch)
        if nbytes == 0:
            raise ValueError("unsupported widths or batch")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        mlp_check(L.mlp_create_ex(warr, self.n, self.max_batch, self.max_train_batch,
                                  C.c_void_p((self.ws.data_ptr() + 255) & ~255), nbytes,
                                  C.byref(h)), "mlp_create_ex")
        self.h = h
        self.P = int(L.mlp_param_count(h))
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().mlp_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_params(self, vec):
        vec = vec.to(device=self.device, dtype=self.torch.float32).contiguous()
        if vec.numel() != self.P:
            raise ValueError(f"expected {self.P} parameters")
        mlp_check(lib().mlp_set_params(self.h, _ptr(vec), _stream(self.torch)), "mlp_set_params")

    def get_params(self):
        out = self.torch.empty(self.P, dtype=self.torch.float32, device=self.device)
        mlp_check(lib().mlp_get_params(self.h, _ptr(out), _stream(self.torch)), "mlp_get_params")
        return out

    def get_grads(self):
        out = self.torch.empty(self.P, dtype=self.torch.float32, device=self.device)
        mlp_check(lib().mlp_get_grads(self.h, _ptr(out), _stream(self.torch)), "mlp_get_grads")
        return out

    def forward(self, x, y=None, keep: bool = False):
        torch = self.torch
        if x.dtype != torch.bfloat16 or x.dim() != 2 or x.shape[1] != self.widths[0] or \
                not x.is_contiguous():
            raise ValueError("x: contiguous bfloat16 [batch][widths[0]]")
        B = x.shape[0]
        if y is None:
            y = torch.empty(B, self.widths[-1], dtype=torch.float32, device=self.device)
        self._x = x  # the backward pass reads the input of the last forward
        mlp_check(lib().mlp_forward(self.h, _ptr(x), _ptr(y), B, int(keep), _stream(torch)),
                  "mlp_forward")
        return y

    def mse(self, y, target, n_valid: int, out=None):
        """Loss into `out` (a float32 device tensor of at least one element; default self.loss)."""
        out = self.loss if out is None else out
        mlp_check(lib().mlp_mse(self.h, _ptr(y), _ptr(target.contiguous()), y.shape[0], int(n_valid),
                                _ptr(out), _stream(self.torch)), "mlp_mse")
        return out

    def backward(self, batch: int):
        mlp_check(lib().mlp_backward(self.h, int(batch), _stream(self.torch)), "mlp_backward")

    def train_step(self, x, target, n_valid: int, lr, beta1=0.9, beta2=0.999, eps=1e-8, y=None,
                   loss=None):
        """forward + MSE + backward + Adam in one library call; returns (y, loss)."""
        torch = self.torch
        B = x.shape[0]
        if x.dtype != torch.bfloat16 or not x.is_contiguous() or x.shape[1] != self.widths[0]:
            raise ValueError("x: contiguous bfloat16 [batch][widths[0]]")
        if y is None:
            y = torch.empty(B, self.widths[-1], dtype=torch.float32, device=self.device)
        loss = self.loss if loss is None else loss
        self._x = x
        mlp_check(lib().mlp_train_step(self.h, _ptr(x), _ptr(target.contiguous()), B, int(n_valid),
                                       float(lr), float(beta1), float(beta2), float(eps), _ptr(y),
                                       _ptr(loss), _stream(torch)), "mlp_train_step")
        return y, loss

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        mlp_check(lib().mlp_adam_step(self.h, float(lr), float(beta1), float(beta2), float(eps),
                                      _stream(self.torch)), "mlp_adam_step")


def gemm_nt(a, b, bias=None, mode: int = 0, z: bool = False):
    """acc = a . b^T (bfloat16 operands): mode 0 -> float32 acc + bias; mode 1 -> (bfloat16
    gelu(acc + bias), float32 acc + bias or None)."""
    torch = _torch()
    M, K = a.shape
    N = b.shape[0]
    if mode == 0:
        c = torch.empty(M, N, dtype=torch.float32, device=a.device)
        zz = None
    else:
        c = torch.empty(M, N, dtype=torch.bfloat16, device=a.device)
        zz = torch.empty(M, N, dtype=torch.float32, device=a.device) if z else None
    mlp_check(lib().mlp_gemm_nt(_ptr(a), a.stride(0), _ptr(b), b.stride(0), _ptr(bias), M, N, K,
                                mode, _ptr(c), N, _ptr(zz), _stream(torch)), "mlp_gemm_nt")
    return c if mode == 0 else (c, zz)
