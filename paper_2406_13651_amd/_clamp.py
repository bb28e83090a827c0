"""ctypes binding of libclamp.so (include/clamp.h), argument marshalling only.

Every function here has the name of the C entry point it calls.  Arrays are
torch tensors on a HIP device; the binding checks their device, dtype,
contiguity and size against the plan (the C ABI only sees pointers), passes
`data_ptr()` and the current stream, and turns a non-OK status into
ClampError.  There is no fallback: without the compiled library, importing
this module raises.
"""

from __future__ import annotations

import ctypes
import sys
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclamp.so")

CLAMP_OK = 0
CLAMP_EINVAL = -1
CLAMP_ESHAPE = -2
CLAMP_EUNSUPPORTED = -3
CLAMP_EDEVICE = -4
CLAMP_ENOMEM = -5

CLAMP_FWD = 0
CLAMP_ADJ = 1
CLAMP_NORMAL = 2

FAULT_NONFINITE = 1
FAULT_RNONPOS = 2
FAULT_GAMMA = 4

DIAG = 8  # doubles of diagnostics per look; the diag array holds looks + 1 rows (the last: summary)
# columns of a look's diag row
DG_GAMMA, DG_DD, DG_AD, DG_H0, DG_H1, DG_MURES, DG_WD, DG_R2 = range(8)
STAGES = 15  # timing stages


class ClampError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("clamp status %d: %s" % (status, msg))
        self.status = status


class clamp_scene(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("looks", ctypes.c_int32), ("pupil_radius", ctypes.c_float),
                ("pupil_mask", ctypes.c_void_p), ("range_support", ctypes.c_int32)]


class clamp_params(ctypes.Structure):
    _fields_ = [("sigma_w2", ctypes.c_float), ("sigma2", ctypes.c_float), ("rho", ctypes.c_float),
                ("beta", ctypes.c_float), ("mu_init_scale", ctypes.c_float),
                ("upsilon", ctypes.POINTER(ctypes.c_float)), ("n_agents", ctypes.c_int32),
                ("r_update", ctypes.c_int32)]


CLAMP_R_QUADRATIC = 0
CLAMP_R_EXACT = 1
R_UPDATES = {"quadratic": CLAMP_R_QUADRATIC, "exact": CLAMP_R_EXACT}


class clamp_fwd_state(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_void_p), ("resid", ctypes.c_void_p), ("r", ctypes.c_void_p),
                ("y_pupil", ctypes.c_void_p), ("ahy2", ctypes.c_void_p)]


class clamp_batch_scene(ctypes.Structure):
    _fields_ = [("params", clamp_params), ("state", clamp_fwd_state), ("w", ctypes.c_void_p),
                ("wbar", ctypes.c_void_p), ("diag", ctypes.c_void_p), ("prior_sigma", ctypes.c_float),
                ("xbar", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libclamp.so is not built (run paper_2406_13651_amd/build.py or "
                          "__graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    sig = {
        "clamp_plan_create": [ctypes.POINTER(clamp_scene), i32, ctypes.POINTER(P)],
        "clamp_plan_destroy": [P],
        "clamp_plan_workspace_size": [P, ctypes.POINTER(ctypes.c_size_t)],
        "clamp_plan_pupil_info": [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(ctypes.c_double)],
        "clamp_plan_pupil_index": [P, i32, ctypes.POINTER(i32)],
        "clamp_aperture_op": [P, i32, i32, P, P, i32, P, P],
        "clamp_fwd_init": [P, i32, ctypes.POINTER(clamp_params), P, ctypes.POINTER(clamp_fwd_state),
                           P, P, P],
        "clamp_fwd_refresh": [P, i32, ctypes.POINTER(clamp_fwd_state), P, P],
        "clamp_fwd_agent_mace": [P, i32, ctypes.POINTER(clamp_params), ctypes.POINTER(clamp_fwd_state),
                                 P, P, P, P, P, P, P, P],
        "clamp_mace_state": [P, i32, ctypes.POINTER(clamp_params), P, P, P, P],
        "clamp_fwd_agent": [P, i32, ctypes.POINTER(clamp_params), ctypes.POINTER(clamp_fwd_state),
                            P, P, P, P, P],
        "clamp_prior_gauss": [P, i32, ctypes.c_float, P, P, P, P],
        "clamp_prior_l21": [P, i32, ctypes.c_float, P, P, P, P],
        "clamp_prior_tv": [P, i32, ctypes.c_float, i32, P, P, P, P],
        "clamp_mace_step": [P, i32, ctypes.POINTER(clamp_params), P, P, P, P, P, P],
        "clamp_mace_step_noalloc": [P, i32, ctypes.POINTER(clamp_params), P, P, P, P, P],
        "clamp_plan_set_timing": [P, i32],
        "clamp_plan_set_timing_stages": [P, ctypes.c_uint32],
        "clamp_batch_workspace_size": [P, ctypes.POINTER(ctypes.c_size_t)],
        "clamp_batch_create": [P, ctypes.POINTER(clamp_batch_scene), P, P, P, ctypes.POINTER(P)],
        "clamp_batch_destroy": [P],
        "clamp_batch_set_iteration": [P, i32, P],
        "clamp_batch_step": [P, P],
        "clamp_batch_set_tiles": [P, i32, i32],
        "clamp_batch_autotune": [P, P, ctypes.POINTER(i32)],
        "clamp_batch_capture": [P, P],
        "clamp_batch_replay": [P, i32, P],
        "clamp_cnn_create": [ctypes.POINTER(P)],
        "clamp_cnn_destroy": [P],
        "clamp_cnn_set_params": [P, ctypes.POINTER(ctypes.c_float)],
        "clamp_cnn_get_params": [P, ctypes.POINTER(ctypes.c_float)],
        "clamp_cnn_workspace_size": [i32, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "clamp_cnn_apply": [P, P, P, i32, i32, i32, i32, i32, P, P],
        "clamp_cnn_grad": [P, P, P, i32, i32, i32, i32, P, P, P, P],
        "clamp_cnn_adam_step": [P, ctypes.c_float, P],
        "clamp_unet_create": [ctypes.POINTER(P)],
        "clamp_unet_destroy": [P],
        "clamp_unet_set_params": [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
        "clamp_unet_get_params": [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
        "clamp_unet_workspace_size": [i32, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "clamp_unet_apply": [P, P, P, i32, i32, i32, i32, i32, P, P],
        "clamp_unet_grad": [P, P, P, i32, i32, i32, i32, P, P, P, P],
        "clamp_unet_adam_step": [P, ctypes.c_float, P],
        "clamp_plan_get_timing": [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    lib.clamp_last_error.argtypes = []
    lib.clamp_last_error.restype = ctypes.c_char_p
    lib.clamp_stage_name.argtypes = [i32]
    lib.clamp_stage_name.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(status):
    if status != CLAMP_OK:
        raise ClampError(status, lib.clamp_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, numel, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must live on the GPU" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < numel:
        raise ValueError("%s holds %d elements, needs %d" % (name, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


class Scene:
    """Host description of one scene (mirrors clamp_scene)."""

    def __init__(self, nx, ny, nz, looks, radius=0.0, mask=None, range_support=0):
        self.nx, self.ny, self.nz, self.looks = int(nx), int(ny), int(nz), int(looks)
        self.radius = float(radius)
        self.range_support = int(range_support)  # 0: per-slice 2D operator; K: 3D operator, K range samples
        self.mask = None
        if mask is not None:
            import numpy as np
            m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8))
            if m.shape != (self.ny, self.nx):
                raise ValueError("mask must be [ny, nx]")
            self.mask = m

    @property
    def n(self):
        return self.nx * self.ny * self.nz


class Plan:
    """Owns a clamp_plan*; released with clamp_plan_destroy."""

    def __init__(self, handle, scenes):
        self.handle = handle
        self.scenes = scenes
        self.info = [clamp_plan_pupil_info(self, i) for i in range(len(scenes))]

    def __del__(self, _finalizing=sys.is_finalizing, _destroy=lib.clamp_plan_destroy):
        h = getattr(self, "handle", None)
        if h and not _finalizing():  # at interpreter exit the process releases everything
            _destroy(h)
            self.handle = None

    def workspace(self, device=None):
        nbytes = clamp_plan_workspace_size(self)
        return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device or "cuda")


def clamp_plan_create(scenes):
    scenes = list(scenes)
    arr = (clamp_scene * len(scenes))()
    for i, s in enumerate(scenes):
        arr[i].nx, arr[i].ny, arr[i].nz, arr[i].looks = s.nx, s.ny, s.nz, s.looks
        arr[i].pupil_radius = s.radius
        arr[i].pupil_mask = s.mask.ctypes.data if s.mask is not None else None
        arr[i].range_support = getattr(s, "range_support", 0)
    h = ctypes.c_void_p()
    _check(lib.clamp_plan_create(arr, len(scenes), ctypes.byref(h)))
    return Plan(h, scenes)


def clamp_plan_workspace_size(plan):
    b = ctypes.c_size_t()
    _check(lib.clamp_plan_workspace_size(plan.handle, ctypes.byref(b)))
    return b.value


def clamp_plan_pupil_info(plan, scene):
    P = ctypes.c_int32()
    B = ctypes.c_int32()
    a = ctypes.c_double()
    _check(lib.clamp_plan_pupil_info(plan.handle, scene, ctypes.byref(P), ctypes.byref(B), ctypes.byref(a)))
    return {"P": P.value, "B": B.value, "alpha": a.value}


def clamp_plan_pupil_index(plan, scene):
    import numpy as np
    P = plan.info[scene]["P"]
    out = np.empty(P, dtype=np.int32)
    _check(lib.clamp_plan_pupil_index(plan.handle, scene, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return out


def clamp_aperture_op(plan, scene, direction, x, out, nbatch, workspace, stream=None):
    s = plan.scenes[scene]
    n = s.n * int(nbatch)
    _check(lib.clamp_aperture_op(plan.handle, scene, int(direction),
                                 _ptr(x, torch.complex64, n, "in"), _ptr(out, torch.complex64, n, "out"),
                                 int(nbatch), _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan),
                                                   "workspace"), _stream(stream)))


def make_params(sigma_w2, sigma2, rho, beta, mu_init_scale, upsilon, r_update="quadratic"):
    """clamp_params; r_update is "quadratic" (App. A) or "exact" (the exact surrogate prox)."""
    ups = (ctypes.c_float * len(upsilon))(*[float(u) for u in upsilon])
    code = R_UPDATES[r_update] if isinstance(r_update, str) else int(r_update)
    p = clamp_params(float(sigma_w2), float(sigma2), float(rho), float(beta), float(mu_init_scale),
                     ctypes.cast(ups, ctypes.POINTER(ctypes.c_float)), len(upsilon), code)
    p._keep = ups
    return p


def _cmp_len(plan, scene):
    """Complex values per look of the compact pupil arrays (resid, y_pupil)."""
    s = plan.scenes[scene]
    P = plan.info[scene]["P"]
    return (s.range_support if getattr(s, "range_support", 0) > 0 else s.nz) * P


def _state(plan, scene, mu, resid, r, n_agents, y_pupil=None, ahy2=None):
    s = plan.scenes[scene]
    st = clamp_fwd_state(_ptr(mu, torch.complex64, s.looks * s.n, "mu").value,
                         _ptr(resid, torch.complex64, s.looks * _cmp_len(plan, scene), "resid").value,
                         _ptr(r, torch.float32, n_agents * s.n, "r").value,
                         None if y_pupil is None else
                         _ptr(y_pupil, torch.complex64, s.looks * _cmp_len(plan, scene), "y_pupil").value,
                         None if ahy2 is None else _ptr(ahy2, torch.float64, s.looks, "ahy2").value)
    return st


def clamp_fwd_init(plan, scene, params, y_full, mu, resid, r, w, workspace, stream=None, y_pupil=None, ahy2=None):
    s = plan.scenes[scene]
    st = _state(plan, scene, mu, resid, r, params.n_agents, y_pupil, ahy2)
    _check(lib.clamp_fwd_init(plan.handle, scene, ctypes.byref(params),
                              _ptr(y_full, torch.complex64, s.looks * s.n, "y_full"), ctypes.byref(st),
                              _ptr(w, torch.float32, params.n_agents * s.n, "w"),
                              _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan), "workspace"),
                              _stream(stream)))


def clamp_fwd_agent(plan, scene, params, mu, resid, r, w, diag, fault, workspace, stream=None, ahy2=None):
    """diag: float64 [(looks + 1) * DIAG] (see include/clamp.h)."""
    s = plan.scenes[scene]
    st = _state(plan, scene, mu, resid, r, s.looks, None, ahy2)
    _check(lib.clamp_fwd_agent(plan.handle, scene, ctypes.byref(params), ctypes.byref(st),
                               _ptr(w, torch.float32, s.looks * s.n, "w"),
                               _ptr(diag, torch.float64, (s.looks + 1) * DIAG, "diag"),
                               _ptr(fault, torch.int32, 1, "fault"),
                               _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan), "workspace"),
                               _stream(stream)))


def clamp_fwd_agent_mace(plan, scene, params, mu, resid, r, w, xbar, wbar, diag, conv_err, fault, workspace,
                         stream=None, ahy2=None):
    """Forward agents with the Mann step fused in (see include/clamp.h for the
    representation of w and xbar)."""
    s = plan.scenes[scene]
    na = params.n_agents
    st = _state(plan, scene, mu, resid, r, na, None, ahy2)
    _check(lib.clamp_fwd_agent_mace(plan.handle, scene, ctypes.byref(params), ctypes.byref(st),
                                    _ptr(w, torch.float32, na * s.n, "w"), _ptr(xbar, torch.float32, s.n, "xbar"),
                                    _ptr(wbar, torch.float32, s.n, "wbar"),
                                    _ptr(diag, torch.float64, (s.looks + 1) * DIAG, "diag"),
                                    _ptr(conv_err, torch.float64, 1, "conv_err"), _ptr(fault, torch.int32, 1, "fault"),
                                    _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan), "workspace"),
                                    _stream(stream)))


def clamp_mace_state(plan, scene, params, w, xbar, out, stream=None):
    s = plan.scenes[scene]
    na = params.n_agents
    _check(lib.clamp_mace_state(plan.handle, scene, ctypes.byref(params), _ptr(w, torch.float32, na * s.n, "w"),
                                _ptr(xbar, torch.float32, s.n, "xbar"), _ptr(out, torch.float32, na * s.n, "out"),
                                _stream(stream)))


def clamp_fwd_refresh(plan, scene, mu, resid, y_pupil, workspace, stream=None):
    s = plan.scenes[scene]
    st = clamp_fwd_state(_ptr(mu, torch.complex64, s.looks * s.n, "mu").value,
                         _ptr(resid, torch.complex64, s.looks * _cmp_len(plan, scene), "resid").value,
                         None,
                         _ptr(y_pupil, torch.complex64, s.looks * _cmp_len(plan, scene), "y_pupil").value,
                         None)
    _check(lib.clamp_fwd_refresh(plan.handle, scene, ctypes.byref(st),
                                 _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan), "workspace"),
                                 _stream(stream)))


def clamp_prior_gauss(plan, scene, sigma_vox, x, out, workspace, stream=None):
    s = plan.scenes[scene]
    _check(lib.clamp_prior_gauss(plan.handle, scene, float(sigma_vox), _ptr(x, torch.float32, s.n, "in"),
                                 _ptr(out, torch.float32, s.n, "out"),
                                 _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan), "workspace"),
                                 _stream(stream)))


def clamp_prior_l21(plan, scene, tau, x, out, workspace, stream=None):
    s = plan.scenes[scene]
    _check(lib.clamp_prior_l21(plan.handle, scene, float(tau), _ptr(x, torch.float32, s.n, "in"),
                               _ptr(out, torch.float32, s.n, "out"),
                               _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan), "workspace"),
                               _stream(stream)))


def clamp_prior_tv(plan, scene, lam, iters, x, out, workspace, stream=None):
    s = plan.scenes[scene]
    _check(lib.clamp_prior_tv(plan.handle, scene, float(lam), int(iters), _ptr(x, torch.float32, s.n, "in"),
                              _ptr(out, torch.float32, s.n, "out"),
                              _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan), "workspace"),
                              _stream(stream)))


def clamp_mace_step(plan, scene, params, w, r, wbar, conv_err, workspace, stream=None):
    s = plan.scenes[scene]
    na = params.n_agents
    _check(lib.clamp_mace_step(plan.handle, scene, ctypes.byref(params), _ptr(w, torch.float32, na * s.n, "w"),
                               _ptr(r, torch.float32, na * s.n, "r"), _ptr(wbar, torch.float32, s.n, "wbar"),
                               _ptr(conv_err, torch.float64, 1, "conv_err"),
                               _ptr(workspace, torch.uint8, clamp_plan_workspace_size(plan), "workspace"),
                               _stream(stream)))


def clamp_mace_step_noalloc(plan, scene, params, w, r, wbar, conv_err, stream=None):
    """clamp_mace_step without a workspace (the library's own 1 MiB scratch)."""
    s = plan.scenes[scene]
    na = params.n_agents
    _check(lib.clamp_mace_step_noalloc(plan.handle, scene, ctypes.byref(params),
                                       _ptr(w, torch.float32, na * s.n, "w"), _ptr(r, torch.float32, na * s.n, "r"),
                                       _ptr(wbar, torch.float32, s.n, "wbar"),
                                       _ptr(conv_err, torch.float64, 1, "conv_err"), _stream(stream)))


def clamp_plan_set_timing(plan, enable):
    _check(lib.clamp_plan_set_timing(plan.handle, 1 if enable else 0))


def clamp_plan_set_timing_stages(plan, names):
    """Time only the named stages (an empty collection turns timing off)."""
    mask = 0
    for name in names:
        idx = [i for i in range(STAGES) if clamp_stage_name(i) == name]
        if not idx:
            raise ValueError("unknown timing stage %r" % name)
        mask |= 1 << idx[0]
    _check(lib.clamp_plan_set_timing_stages(plan.handle, ctypes.c_uint32(mask)))


def clamp_plan_get_timing(plan):
    """{stage name: (total ms, launches)} of the records since the last call."""
    ms = (ctypes.c_double * STAGES)()
    cnt = (ctypes.c_int32 * STAGES)()
    _check(lib.clamp_plan_get_timing(plan.handle, ms, cnt))
    return {clamp_stage_name(i): (ms[i], cnt[i]) for i in range(STAGES) if cnt[i] > 0}


def clamp_stage_name(stage):
    return lib.clamp_stage_name(int(stage)).decode()


# -- batches ---------------------------------------------------------------

def clamp_batch_workspace_size(plan):
    b = ctypes.c_size_t()
    _check(lib.clamp_batch_workspace_size(plan.handle, ctypes.byref(b)))
    return b.value


class Batch:
    """Owns a clamp_batch*; released with clamp_batch_destroy."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep

    def __del__(self, _finalizing=sys.is_finalizing, _destroy=lib.clamp_batch_destroy):
        h = getattr(self, "handle", None)
        if h and not _finalizing():  # at interpreter exit the process releases everything
            _destroy(h)
            self.handle = None


def clamp_batch_create(plan, scenes, fault, conv_err, workspace):
    """scenes: list of dicts with params (clamp_params), mu, resid, r, w, wbar,
    diag (tensors), prior_sigma and optional ahy2 and xbar (tensors; xbar on
    every scene selects the fused Mann step)."""
    arr = (clamp_batch_scene * len(scenes))()
    for i, sc in enumerate(scenes):
        s = plan.scenes[i]
        na = sc["params"].n_agents
        st = _state(plan, i, sc["mu"], sc["resid"], sc["r"], na, None, sc.get("ahy2"))
        arr[i].params = sc["params"]
        arr[i].state = st
        arr[i].w = _ptr(sc["w"], torch.float32, na * s.n, "w").value
        arr[i].wbar = _ptr(sc["wbar"], torch.float32, s.n, "wbar").value
        arr[i].diag = _ptr(sc["diag"], torch.float64, (s.looks + 1) * DIAG, "diag").value
        arr[i].prior_sigma = float(sc.get("prior_sigma", 1.0))
        xb = sc.get("xbar")
        arr[i].xbar = None if xb is None else _ptr(xb, torch.float32, s.n, "xbar").value
    h = ctypes.c_void_p()
    _check(lib.clamp_batch_create(plan.handle, arr, _ptr(fault, torch.int32, 1, "fault"),
                                  _ptr(conv_err, torch.float64, len(scenes), "conv_err"),
                                  _ptr(workspace, torch.uint8, clamp_batch_workspace_size(plan), "workspace"),
                                  ctypes.byref(h)))
    return Batch(h, [sc["params"] for sc in scenes])


def clamp_batch_set_iteration(batch, done, stream=None):
    _check(lib.clamp_batch_set_iteration(batch.handle, int(done), _stream(stream)))


def clamp_batch_step(batch, stream=None):
    _check(lib.clamp_batch_step(batch.handle, _stream(stream)))


def clamp_batch_set_tiles(batch, row_blocks_per_cu, col_blocks_per_cu):
    _check(lib.clamp_batch_set_tiles(batch.handle, int(row_blocks_per_cu), int(col_blocks_per_cu)))


def clamp_batch_autotune(batch, stream=None):
    out = (ctypes.c_int32 * 2)()
    _check(lib.clamp_batch_autotune(batch.handle, _stream(stream), out))
    return {"row_blocks_per_cu": out[0], "col_blocks_per_cu": out[1]}


def clamp_batch_capture(batch, stream):
    _check(lib.clamp_batch_capture(batch.handle, _stream(stream)))


def clamp_batch_replay(batch, iters, stream):
    _check(lib.clamp_batch_replay(batch.handle, int(iters), _stream(stream)))


# -- learned prior (CNN) ------------------------------------------------------

CNN_PARAMS = 167841


class Cnn:
    """Owns a clamp_cnn*; released with clamp_cnn_destroy."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib.clamp_cnn_create(ctypes.byref(h)))
        self.handle = h

    def __del__(self, _finalizing=sys.is_finalizing, _destroy=lib.clamp_cnn_destroy):
        h = getattr(self, "handle", None)
        if h and not _finalizing():  # at interpreter exit the process releases everything
            _destroy(h)
            self.handle = None


def clamp_cnn_create():
    return Cnn()


def clamp_cnn_set_params(cnn, params):
    import numpy as np
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    if p.size != CNN_PARAMS:
        raise ValueError("expected %d parameters" % CNN_PARAMS)
    _check(lib.clamp_cnn_set_params(cnn.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))


def clamp_cnn_get_params(cnn):
    import numpy as np
    p = np.empty(CNN_PARAMS, dtype=np.float32)
    _check(lib.clamp_cnn_get_params(cnn.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return p


def clamp_cnn_workspace_size(nvol, nz, ny, nx, train):
    b = ctypes.c_size_t()
    _check(lib.clamp_cnn_workspace_size(int(nvol), int(nz), int(ny), int(nx), 1 if train else 0, ctypes.byref(b)))
    return b.value


def clamp_cnn_apply(cnn, x, out, normalize, workspace, stream=None):
    """x, out: float32 [nvol, nz, ny, nx] (or [nz, ny, nx]) on the GPU."""
    shape = tuple(x.shape) if x.dim() == 4 else (1,) + tuple(x.shape)
    nvol, nz, ny, nx = shape
    n = nvol * nz * ny * nx
    _check(lib.clamp_cnn_apply(cnn.handle, _ptr(x, torch.float32, n, "x"), _ptr(out, torch.float32, n, "out"),
                               nvol, nz, ny, nx, 1 if normalize else 0,
                               _ptr(workspace, torch.uint8, clamp_cnn_workspace_size(nvol, nz, ny, nx, False),
                                    "workspace"), _stream(stream)))


def clamp_cnn_grad(cnn, x, target, loss, workspace, grad=None, stream=None):
    nvol, nz, ny, nx = x.shape
    n = nvol * nz * ny * nx
    g = _ptr(grad, torch.float32, CNN_PARAMS, "grad") if grad is not None else None
    _check(lib.clamp_cnn_grad(cnn.handle, _ptr(x, torch.float32, n, "x"), _ptr(target, torch.float32, n, "target"),
                              nvol, nz, ny, nx, _ptr(loss, torch.float64, 1, "loss"), g,
                              _ptr(workspace, torch.uint8, clamp_cnn_workspace_size(nvol, nz, ny, nx, True),
                                   "workspace"), _stream(stream)))


def clamp_cnn_adam_step(cnn, lr, stream=None):
    _check(lib.clamp_cnn_adam_step(cnn.handle, float(lr), _stream(stream)))


# -- U-Net prior --------------------------------------------------------------

UNET_PARAMS = 331297
UNET_STATS = 12 * 2 * 32


class Unet:
    """Owns a clamp_unet*; released with clamp_unet_destroy."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib.clamp_unet_create(ctypes.byref(h)))
        self.handle = h

    def __del__(self, _finalizing=sys.is_finalizing, _destroy=lib.clamp_unet_destroy):
        h = getattr(self, "handle", None)
        if h and not _finalizing():  # at interpreter exit the process releases everything
            _destroy(h)
            self.handle = None


def clamp_unet_create():
    return Unet()


def clamp_unet_set_params(unet, params, stats=None):
    import numpy as np
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    if p.size != UNET_PARAMS:
        raise ValueError("expected %d parameters" % UNET_PARAMS)
    sp = None
    if stats is not None:
        st = np.ascontiguousarray(np.asarray(stats, dtype=np.float32))
        if st.size != UNET_STATS:
            raise ValueError("expected %d running statistics" % UNET_STATS)
        sp = st.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    _check(lib.clamp_unet_set_params(unet.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), sp))


def clamp_unet_get_params(unet):
    """(parameters, running statistics) as float32 numpy arrays."""
    import numpy as np
    p = np.empty(UNET_PARAMS, dtype=np.float32)
    st = np.empty(UNET_STATS, dtype=np.float32)
    _check(lib.clamp_unet_get_params(unet.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     st.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return p, st


def clamp_unet_workspace_size(nvol, nz, ny, nx, train):
    b = ctypes.c_size_t()
    _check(lib.clamp_unet_workspace_size(int(nvol), int(nz), int(ny), int(nx), 1 if train else 0, ctypes.byref(b)))
    return b.value


def clamp_unet_apply(unet, x, out, normalize, workspace, stream=None):
    """x, out: float32 [nvol, nz, ny, nx] (or [nz, ny, nx]) on the GPU."""
    shape = tuple(x.shape) if x.dim() == 4 else (1,) + tuple(x.shape)
    nvol, nz, ny, nx = shape
    n = nvol * nz * ny * nx
    _check(lib.clamp_unet_apply(unet.handle, _ptr(x, torch.float32, n, "x"), _ptr(out, torch.float32, n, "out"),
                                nvol, nz, ny, nx, 1 if normalize else 0,
                                _ptr(workspace, torch.uint8, clamp_unet_workspace_size(nvol, nz, ny, nx, False),
                                     "workspace"), _stream(stream)))


def clamp_unet_grad(unet, x, target, loss, workspace, grad=None, stream=None):
    nvol, nz, ny, nx = x.shape
    n = nvol * nz * ny * nx
    g = _ptr(grad, torch.float32, UNET_PARAMS, "grad") if grad is not None else None
    _check(lib.clamp_unet_grad(unet.handle, _ptr(x, torch.float32, n, "x"), _ptr(target, torch.float32, n, "target"),
                               nvol, nz, ny, nx, _ptr(loss, torch.float64, 1, "loss"), g,
                               _ptr(workspace, torch.uint8, clamp_unet_workspace_size(nvol, nz, ny, nx, True),
                                    "workspace"), _stream(stream)))


def clamp_unet_adam_step(unet, lr, stream=None):
    _check(lib.clamp_unet_adam_step(unet.handle, float(lr), _stream(stream)))
