"""MI355X-native implicit Discrete Elastic Rods (DisMech, arXiv 2311.18126).

Thin ctypes binding of libdmrod.so (include/dmrod.h).  The binding only marshals
arguments: every part of the time step runs in the library's HIP kernels.  Importing
this package never builds or falls back to anything; `lib()` raises if the shared
library is missing or cannot be loaded.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdmrod.so")

DM_OK = 0
DM_NOT_CONVERGED = 1
DM_ERR_INVALID_ARG = -1
DM_ERR_STATE = -2
DM_ERR_HIP = -3
DM_ERR_OOM = -4
DM_ERR_SINGULAR = -5
DM_ERR_UNSUPPORTED = -6

NET_IN = 26     # warm-start features per row (checked against the library when a network is made)
DM_MLP_NOALLOC_MAX_ROWS = 2048     # rows of dm_mlp_forward_noalloc's static activation buffer


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class DmConfig(ctypes.Structure):
    _fields_ = [("gravity", c_double * 3), ("newton_tol", c_double), ("floor_factor", c_double), ("max_iter", c_int),
                ("line_search", c_int), ("floor_contact", c_int), ("floor_z", c_double),
                ("delta", c_double), ("nu", c_double), ("mu", c_double), ("k_contact", c_double),
                ("damping", c_double), ("device", c_int), ("stream", c_void_p), ("block_size", c_int),
                ("warm_max_iter", c_int), ("use_graphs", c_int), ("alloc", ALLOC_FN), ("free_", FREE_FN),
                ("alloc_ctx", c_void_p)]


class DmStats(ctypes.Structure):
    _fields_ = [("steps_done", c_int), ("newton_iters", c_int), ("status", c_int), ("floor_steps", c_int),
                ("fallbacks", c_int), ("halvings", c_int), ("residual", c_double), ("floor_residual_max", c_double),
                ("floor_estimate", c_double)]


_DP = POINTER(c_double)
_IP = POINTER(c_int)
_SIGS = {
    "dm_config_default": (None, [POINTER(DmConfig)]),
    "dm_create": (c_int, [POINTER(DmConfig), POINTER(c_void_p)]),
    "dm_add_rod": (c_int, [c_void_p, c_int, _DP, c_double, c_double, c_double, c_double, _IP]),
    "dm_add_joint": (c_int, [c_void_p, c_int, c_int, c_int, c_int]),
    "dm_fix_nodes": (c_int, [c_void_p, c_int, _IP, c_int]),
    "dm_fix_edges": (c_int, [c_void_p, c_int, _IP, c_int]),
    "dm_set_natural_curvature": (c_int, [c_void_p, c_int, _DP]),
    "dm_set_actuation_sine": (c_int, [c_void_p, c_int, c_double, c_double, c_double]),
    "dm_set_external_load": (c_int, [c_void_p, c_int, _DP, _DP]),
    "dm_finalize": (c_int, [c_void_p]),
    "dm_step": (c_int, [c_void_p, c_double, c_int, POINTER(DmStats)]),
    "dm_num_systems": (c_int, [c_void_p]),
    "dm_rod_system": (c_int, [c_void_p, c_int]),
    "dm_num_rods": (c_int, [c_void_p]),
    "dm_rod_nodes": (c_int, [c_void_p, c_int]),
    "dm_get_rod_state": (c_int, [c_void_p, c_int, _DP, _DP, _DP, _DP]),
    "dm_set_rod_state": (c_int, [c_void_p, c_int, _DP, _DP, _DP, _DP]),
    "dm_num_nodes": (c_int, [c_void_p]),
    "dm_num_edges": (c_int, [c_void_p]),
    "dm_node_index": (c_int, [c_void_p, c_int, c_int]),
    "dm_edge_index": (c_int, [c_void_p, c_int, c_int]),
    "dm_get_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "dm_set_state": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "dm_checkpoint_size": (c_size_t, [c_void_p]),
    "dm_save_checkpoint": (c_int, [c_void_p, c_void_p, c_int]),
    "dm_load_checkpoint": (c_int, [c_void_p, c_void_p, c_int]),
    "dm_set_natural_curvature_all": (c_int, [c_void_p, c_void_p, c_int]),
    "dm_rollout": (c_int, [c_void_p, c_double, c_int, c_int, c_void_p, c_int]),
    "dm_adjoint": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int]),
    "dm_fit_natural_curvature": (c_int, [c_void_p, c_double, c_int, c_int, c_void_p, c_int, c_double, c_double,
                                         c_int, c_void_p, c_int, _DP, POINTER(c_int)]),
    "dm_limb_curvatures": (c_int, [c_void_p, _DP]),
    "dm_limb_curvature_gradient": (c_int, [c_void_p, c_double, _DP, _DP]),
    "dm_fit_limb_curvatures": (c_int, [c_void_p, c_double, c_int, c_int, _DP, c_double, c_double, c_int, _DP,
                                       _IP, _DP]),
    "dm_mlp_num_params": (c_size_t, []),
    "dm_mlp_num_inputs": (c_int, []),
    "dm_mlp_create": (c_int, [c_int, c_void_p, c_int, POINTER(c_void_p)]),
    "dm_mlp_set_params": (c_int, [c_void_p, c_void_p, c_int]),
    "dm_mlp_get_params": (c_int, [c_void_p, c_void_p, c_int]),
    "dm_mlp_set_normalisation": (c_int, [c_void_p, _DP, _DP, _DP]),
    "dm_mlp_get_normalisation": (c_int, [c_void_p, _DP, _DP, _DP]),
    "dm_mlp_fit_normalisation": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    "dm_mlp_forward": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    "dm_mlp_forward_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    "dm_mlp_gradients": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, _DP]),
    "dm_mlp_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_float, _DP]),
    "dm_mlp_train_epoch": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_float, _DP]),
    "dm_mlp_last_error": (c_char_p, []),
    "dm_contact_create": (c_int, [c_int, c_void_p, c_int, c_int, _IP, _IP, _DP, _DP, _DP, c_int, _IP, c_double, c_int,
                                  POINTER(c_void_p)]),
    "dm_contact_find": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_int)]),
    "dm_contact_terms": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double, c_double, c_double, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dm_contact_last_ms": (c_double, [c_void_p, c_int]),
    "dm_contact_last_error": (c_char_p, []),
    "dm_contact_destroy": (None, [c_void_p]),
    "dm_mlp_destroy": (None, [c_void_p]),
    "dm_ws_rows": (c_int, [c_void_p]),
    "dm_ws_features": (c_int, [c_void_p, c_void_p]),
    "dm_ws_targets": (c_int, [c_void_p, c_void_p, c_double, c_void_p]),
    "dm_set_warm_start": (c_int, [c_void_p, c_void_p, c_int]),
    "dm_set_integrator": (c_int, [c_void_p, c_int]),
    "dm_set_self_contact": (c_int, [c_void_p, c_double, c_double, c_double, c_double]),
    "dm_set_adaptive": (c_int, [c_void_p, c_int]),
    "dm_ws_predict": (c_int, [c_void_p, c_double, c_void_p, c_int]),
    "dm_autotune": (c_int, [c_void_p, c_double, c_int, c_char_p, POINTER(c_int)]),
    "dm_time": (c_double, [c_void_p]),
    "dm_last_kernel_ms": (c_double, [c_void_p]),
    "dm_block_size": (c_int, [c_void_p]),
    "dm_last_error": (c_char_p, []),
    "dm_destroy": (None, [c_void_p]),
}

_lib = None


def lib():
    """Load libdmrod.so (built by paper_2311_18126_amd.build); raise if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_18126_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DmError(RuntimeError):
    def __init__(self, status, where):
        # each part of the library keeps its own last message
        src = (lib().dm_mlp_last_error if where.startswith("dm_mlp")
               else lib().dm_contact_last_error if where.startswith("dm_contact") else lib().dm_last_error)
        msg = src().decode(errors="replace")
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def _check(status, where, allow=(DM_OK,)):
    if status not in allow:
        raise DmError(status, where)
    return status


def _dp(a):
    return a.ctypes.data_as(_DP)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _sized(a, n, what):
    """float64 contiguous host copy of a, which must hold exactly n values (the library reads
    the sizes it is told, so a short array is refused here)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != n:
        raise ValueError(f"{what} must hold {n} values, got {a.size}")
    return a


def _device_sized(t, n, what):
    """A float64 contiguous device tensor of at least n values."""
    import torch
    if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{what} must be a contiguous float64 device tensor of at least {n} values")
    return t


def _torch_cuda():
    try:
        import torch
        return torch.cuda.is_available()
    except ImportError:
        return False


def _torch_hooks(device, stream):
    """Allocator callbacks of dm_config backed by PyTorch's caching allocator on the given
    device and stream (an int hipStream_t or None for the null stream).  Returns the two ctypes
    callbacks; the caller keeps them alive while the simulation exists."""
    import torch
    sptr = int(stream) if stream else 0

    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, sptr)
        except Exception:          # out of memory: the library reports DM_ERR_OOM
            return None

    def free(ptr, ctx):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:          # interpreter shutdown: nothing left to return the pages to
            pass
    return ALLOC_FN(alloc), FREE_FN(free)


class Sim:
    """One dm_sim.  Build with add_rod / add_joint / ..., then finalize() and step()."""

    def __init__(self, gravity=(0.0, 0.0, -9.81), newton_tol=1e-9, max_iter=50, line_search=False,
                 floor=None, damping=0.0, device=0, stream=None, block_size=0, floor_factor=1.0,
                 warm_max_iter=0, use_graphs=True, torch_memory=True):
        """torch_memory: obtain every device buffer of the simulation from PyTorch's caching
        allocator (dm_config.alloc / free_) instead of hipMalloc."""
        L = lib()
        cfg = DmConfig()
        L.dm_config_default(ctypes.byref(cfg))
        for i in range(3):
            cfg.gravity[i] = float(gravity[i])
        cfg.newton_tol = float(newton_tol)
        cfg.floor_factor = float(floor_factor)
        cfg.max_iter = int(max_iter)
        cfg.line_search = int(bool(line_search))
        if floor is not None:
            cfg.floor_contact = 1
            cfg.floor_z = float(floor["z"])
            cfg.delta = float(floor["delta"])
            cfg.nu = float(floor["nu"])
            cfg.mu = float(floor["mu"])
            cfg.k_contact = float(floor["k_c"])
        cfg.damping = float(damping)
        cfg.device = int(device)
        cfg.stream = stream
        cfg.block_size = int(block_size)
        cfg.warm_max_iter = int(warm_max_iter)
        cfg.use_graphs = int(bool(use_graphs))
        self._hooks = None
        if torch_memory and _torch_cuda():
            # without a visible GPU no hook is set and dm_create itself reports DM_ERR_HIP
            self._hooks = _torch_hooks(int(device), stream)
            cfg.alloc, cfg.free_ = self._hooks
        h = c_void_p()
        _check(L.dm_create(ctypes.byref(cfg), ctypes.byref(h)), "dm_create")
        self._h = h
        self.cfg = cfg

    def close(self):
        if getattr(self, "_h", None):
            lib().dm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- construction -------------------------------------------------------
    def add_rod(self, x0, radius, E, poisson=0.5, density=1000.0):
        x0 = _f64(x0)
        if x0.ndim != 2 or x0.shape[1] != 3:
            raise ValueError("x0 must have shape (n_nodes, 3)")
        rid = c_int()
        _check(lib().dm_add_rod(self._h, x0.shape[0], _dp(x0), radius, E, poisson, density, ctypes.byref(rid)),
               "dm_add_rod")
        return rid.value

    def add_joint(self, rod_a, node_a, rod_b, node_b):
        _check(lib().dm_add_joint(self._h, rod_a, node_a, rod_b, node_b), "dm_add_joint")

    def fix_nodes(self, rod, nodes):
        a = np.ascontiguousarray(nodes, dtype=np.int32)
        _check(lib().dm_fix_nodes(self._h, rod, a.ctypes.data_as(_IP), a.size), "dm_fix_nodes")

    def fix_edges(self, rod, edges):
        a = np.ascontiguousarray(edges, dtype=np.int32)
        _check(lib().dm_fix_edges(self._h, rod, a.ctypes.data_as(_IP), a.size), "dm_fix_edges")

    def set_natural_curvature(self, rod, kbar):
        k = _sized(kbar, 2 * max(lib().dm_rod_nodes(self._h, rod) - 2, 0), "kbar")
        _check(lib().dm_set_natural_curvature(self._h, rod, _dp(k)), "dm_set_natural_curvature")

    def set_actuation_sine(self, rod, A, f, phi):
        _check(lib().dm_set_actuation_sine(self._h, rod, A, f, phi), "dm_set_actuation_sine")

    def set_external_load(self, rod, force=None, moment=None):
        n = lib().dm_rod_nodes(self._h, rod)
        fp = _sized(force, 3 * n, "force") if force is not None else None
        mp = _sized(moment, max(n - 1, 0), "moment") if moment is not None else None
        _check(lib().dm_set_external_load(self._h, rod, _dp(fp) if fp is not None else None,
                                          _dp(mp) if mp is not None else None), "dm_set_external_load")

    def finalize(self):
        _check(lib().dm_finalize(self._h), "dm_finalize")

    # -- stepping -----------------------------------------------------------
    def step(self, dt, nsteps=1, allow_failure=False):
        """Advance all systems; returns a structured numpy array of per-system statistics."""
        n = lib().dm_num_systems(self._h)
        st = (DmStats * max(n, 1))()
        s = lib().dm_step(self._h, float(dt), int(nsteps), st)
        if not allow_failure:
            _check(s, "dm_step")
        self.last_status = s
        out = np.zeros(n, dtype=[("steps", np.int32), ("iters", np.int32), ("status", np.int32),
                                 ("floor_steps", np.int32), ("fallbacks", np.int32), ("halvings", np.int32),
                                 ("residual", np.float64), ("floor_residual_max", np.float64),
                                 ("floor_estimate", np.float64)])
        for i in range(n):
            out[i] = (st[i].steps_done, st[i].newton_iters, st[i].status, st[i].floor_steps, st[i].fallbacks,
                      st[i].halvings, st[i].residual, st[i].floor_residual_max, st[i].floor_estimate)
        return out

    def set_self_contact(self, delta, k_c, mu=0.0, nu=1e-3):
        """Edge-edge self-contact of every rod inside step() (dm_set_self_contact); k_c = 0
        turns it off."""
        _check(lib().dm_set_self_contact(self._h, float(delta), float(k_c), float(mu), float(nu)),
               "dm_set_self_contact")

    def set_integrator(self, scheme):
        """Time integrator of step(): "euler" (backward Euler, the default) or "midpoint"
        (implicit midpoint); see dm_set_integrator."""
        code = {"euler": 0, "midpoint": 1}.get(scheme)
        if code is None:
            raise ValueError(f"unknown integrator {scheme!r}")
        _check(lib().dm_set_integrator(self._h, code), "dm_set_integrator")

    def set_adaptive(self, max_halvings):
        """Adaptive time stepping of step(): a step whose Newton solve fails is redone as two
        half steps, recursively, at most max_halvings levels deep (0: off); see dm_set_adaptive."""
        _check(lib().dm_set_adaptive(self._h, int(max_halvings)), "dm_set_adaptive")

    # -- state --------------------------------------------------------------
    @property
    def num_systems(self):
        return lib().dm_num_systems(self._h)

    @property
    def num_nodes(self):
        return lib().dm_num_nodes(self._h)

    @property
    def num_edges(self):
        return lib().dm_num_edges(self._h)

    def rod_system(self, rod):
        return lib().dm_rod_system(self._h, rod)

    def rod_state(self, rod):
        n = lib().dm_rod_nodes(self._h, rod)
        x, v = np.zeros((n, 3)), np.zeros((n, 3))
        th, om = np.zeros(n - 1), np.zeros(n - 1)
        _check(lib().dm_get_rod_state(self._h, rod, _dp(x), _dp(th), _dp(v), _dp(om)), "dm_get_rod_state")
        return x, th, v, om

    def set_rod_state(self, rod, x=None, theta=None, v=None, theta_dot=None):
        n = lib().dm_rod_nodes(self._h, rod)
        arrs = [None if a is None else _sized(a, m, w) for a, m, w in
                ((x, 3 * n, "x"), (theta, n - 1, "theta"), (v, 3 * n, "v"), (theta_dot, n - 1, "theta_dot"))]
        args = [(_dp(a) if a is not None else None) for a in arrs]
        _check(lib().dm_set_rod_state(self._h, rod, *args), "dm_set_rod_state")

    def state(self):
        """Bulk state in the library's global numbering (host numpy arrays)."""
        x, v = np.zeros((self.num_nodes, 3)), np.zeros((self.num_nodes, 3))
        th, om = np.zeros(self.num_edges), np.zeros(self.num_edges)
        _check(lib().dm_get_state(self._h, x.ctypes.data, th.ctypes.data, v.ctypes.data, om.ctypes.data, 0),
               "dm_get_state")
        return x, th, v, om

    def set_state(self, x=None, theta=None, v=None, theta_dot=None):
        """Set the bulk state (global numbering, host arrays; None leaves a part unchanged)."""
        args = []
        for a, shp in ((x, (self.num_nodes, 3)), (theta, (self.num_edges,)), (v, (self.num_nodes, 3)),
                       (theta_dot, (self.num_edges,))):
            args.append(None if a is None else _f64(a, shp))
        ptr = [a.ctypes.data if a is not None else None for a in args]
        _check(lib().dm_set_state(self._h, ptr[0], ptr[1], ptr[2], ptr[3], 0), "dm_set_state")

    def state_torch(self, device="cuda"):
        """Bulk state copied device-to-device into new torch tensors."""
        import torch
        x = torch.empty((self.num_nodes, 3), dtype=torch.float64, device=device)
        v = torch.empty_like(x)
        th = torch.empty(self.num_edges, dtype=torch.float64, device=device)
        om = torch.empty_like(th)
        _check(lib().dm_get_state(self._h, x.data_ptr(), th.data_ptr(), v.data_ptr(), om.data_ptr(), 1),
               "dm_get_state")
        return x, th, v, om

    def node_index(self, rod, node):
        return lib().dm_node_index(self._h, rod, node)

    def edge_index(self, rod, edge):
        return lib().dm_edge_index(self._h, rod, edge)

    def checkpoint(self):
        n = lib().dm_checkpoint_size(self._h)
        buf = np.zeros(n)
        _check(lib().dm_save_checkpoint(self._h, buf.ctypes.data, 0), "dm_save_checkpoint")
        return buf

    def restore(self, buf):
        """Load a checkpoint from a host array or a device tensor (checkpoint_torch)."""
        n = lib().dm_checkpoint_size(self._h)
        if _is_cuda_tensor(buf):
            _device_sized(buf, n, "checkpoint")
            _check(lib().dm_load_checkpoint(self._h, buf.data_ptr(), 1), "dm_load_checkpoint")
            return
        buf = _sized(buf, n, "checkpoint")
        _check(lib().dm_load_checkpoint(self._h, buf.ctypes.data, 0), "dm_load_checkpoint")

    def checkpoint_torch(self, device="cuda"):
        import torch
        buf = torch.empty(lib().dm_checkpoint_size(self._h), dtype=torch.float64, device=device)
        _check(lib().dm_save_checkpoint(self._h, buf.data_ptr(), 1), "dm_save_checkpoint")
        return buf

    def autotune(self, dt, trial_steps=3, cache=None):
        """Pick the step kernel's workgroup size by timing (cached in the file `cache`)."""
        b = c_int()
        _check(lib().dm_autotune(self._h, float(dt), int(trial_steps), cache.encode() if cache else None,
                                 ctypes.byref(b)), "dm_autotune")
        return b.value

    @property
    def ws_rows(self):
        """Rows of the warm-start feature matrix (one per rod node)."""
        return lib().dm_ws_rows(self._h)

    def ws_features(self, out):
        """Raw warm-start features of every row at the current state into `out`, a float64
        device tensor (ws_rows, NET_IN)."""
        _check(lib().dm_ws_features(self._h, out.data_ptr()), "dm_ws_features")
        return out

    def ws_targets(self, features_prev, dt, out):
        """Targets dt (v_{n+1} - v_n - a_n - j_n) after a step, from the step-start features,
        into `out` (float64 device tensor (ws_rows, 3))."""
        _check(lib().dm_ws_targets(self._h, features_prev.data_ptr(), dt, out.data_ptr()), "dm_ws_targets")
        return out

    def ws_predict(self, dt, out=None):
        """Guessed displacement of every feature row for a step of `dt` under the current warm
        mode, into `out` (float64 device tensor (ws_rows, 3)), or returned as a numpy array."""
        if out is not None:
            _check(lib().dm_ws_predict(self._h, dt, out.data_ptr(), 1), "dm_ws_predict")
            return out
        h = np.zeros((self.ws_rows, 3))
        _check(lib().dm_ws_predict(self._h, dt, h.ctypes.data, 0), "dm_ws_predict")
        return h

    def set_warm_start(self, net=None, mode=None):
        """Warm start of step(): None/0 off, 1 explicit predictor x_n + dt v_n, 3 the
        second-order extrapolation x_n + dt (v_n + a_n), 4 the third-order one
        x_n + dt (v_n + a_n + j_n), 2 the network `net` on top of the third-order one."""
        if mode is None:
            mode = 0 if net is None else 2
        _check(lib().dm_set_warm_start(self._h, net._h if net is not None else None, mode), "dm_set_warm_start")
        self._ws_net = net

    @property
    def num_rods(self):
        return lib().dm_num_rods(self._h)

    def rod_nodes(self, rod):
        return lib().dm_rod_nodes(self._h, rod)

    @property
    def kbar_size(self):
        """Length of the concatenated natural-curvature vector (2 (N_r - 2) per rod)."""
        return sum(2 * max(self.rod_nodes(r) - 2, 0) for r in range(self.num_rods))

    def set_natural_curvature_all(self, kbar):
        """Every rod's natural curvature [N_r-2][2] (1/m), concatenated in rod order; a host
        array or a float64 device tensor."""
        if _is_cuda_tensor(kbar):
            k = _device_sized(kbar.detach().contiguous(), self.kbar_size, "kbar")
            _check(lib().dm_set_natural_curvature_all(self._h, k.data_ptr(), 1), "dm_set_natural_curvature_all")
        else:
            k = _sized(kbar, self.kbar_size, "kbar")
            _check(lib().dm_set_natural_curvature_all(self._h, k.ctypes.data, 0), "dm_set_natural_curvature_all")

    def limb_curvatures(self):
        """Every rod's limb curvature (1/m): see dm_limb_curvatures."""
        k = np.zeros(self.num_rods)
        _check(lib().dm_limb_curvatures(self._h, _dp(k)), "dm_limb_curvatures")
        return k

    def limb_curvature_gradient(self, dt, weights):
        """d(sum w kappa)/d kbar per rod at the current state: see dm_limb_curvature_gradient."""
        w = _sized(weights, self.num_rods, "weights")
        g = np.zeros(self.num_rods)
        _check(lib().dm_limb_curvature_gradient(self._h, float(dt), _dp(w), _dp(g)), "dm_limb_curvature_gradient")
        return g

    def fit_limb_curvatures(self, dt, n_settle, targets, alpha0=0.1, tol=1e-3, max_iter=200):
        """Alg. 1 over target limb curvatures (n_configs, n_rods); returns the fitted natural
        curvature after each configuration (n_configs, n_rods), the gradient steps and the last
        loss of each configuration and system (n_configs, n_systems)."""
        t = _f64(targets)
        if t.ndim != 2 or t.shape[1] != self.num_rods:
            raise ValueError(f"targets must have shape (n_configs, {self.num_rods})")
        nc, ns = t.shape[0], self.num_systems
        traj = np.zeros((nc, self.num_rods))
        steps = np.zeros((nc, ns), dtype=np.int32)
        losses = np.zeros((nc, ns))
        _check(lib().dm_fit_limb_curvatures(self._h, float(dt), int(n_settle), nc, _dp(t), float(alpha0), float(tol),
                                            int(max_iter), _dp(traj), steps.ctypes.data_as(_IP), _dp(losses)),
               "dm_fit_limb_curvatures")
        return traj, steps, losses

    def rollout(self, dt, nsteps, ckpt_every=20, out=None):
        """nsteps steps with a checkpoint every ckpt_every steps, for adjoint(); returns the tip
        (last node) of every rod after every step, (nsteps, n_rods, 3), into `out` (a float64
        device tensor) or a new host array."""
        if out is not None:
            _device_sized(out, int(nsteps) * self.num_rods * 3, "out")
            _check(lib().dm_rollout(self._h, dt, nsteps, ckpt_every, out.data_ptr(), 1), "dm_rollout")
            self._roll_steps = int(nsteps)
            return out
        tips = np.zeros((nsteps, self.num_rods, 3))
        _check(lib().dm_rollout(self._h, dt, nsteps, ckpt_every, tips.ctypes.data, 0), "dm_rollout")
        self._roll_steps = int(nsteps)
        return tips

    def adjoint(self, dL_dtips, out=None):
        """Gradient of a tip-trajectory loss with respect to the concatenated natural curvature,
        from dL/dtips of the last rollout (host array or device tensor); into `out` (float64
        device tensor) or a new host array."""
        # sizes are checked against the last rollout; without one the library reports the
        # missing rollout (DM_ERR_STATE) before reading anything
        steps = getattr(self, "_roll_steps", None)
        n = (steps or 0) * self.num_rods * 3
        if _is_cuda_tensor(dL_dtips):
            g = dL_dtips.detach().contiguous()
            if steps is not None:
                _device_sized(g, n, "dL_dtips")
            src, on_dev = g.data_ptr(), 1
        else:
            g = _f64(dL_dtips) if steps is None else _sized(dL_dtips, n, "dL_dtips")
            src, on_dev = g.ctypes.data, 0
        if out is not None:
            _device_sized(out, self.kbar_size, "out")
            _check(lib().dm_adjoint(self._h, src, on_dev, out.data_ptr(), 1), "dm_adjoint")
            return out
        res = np.zeros(self.kbar_size)
        _check(lib().dm_adjoint(self._h, src, on_dev, res.ctypes.data, 0), "dm_adjoint")
        return res

    def fit_natural_curvature(self, dt, nsteps, target_tips, kbar0=None, alpha0=0.1, tol=0.0, max_iter=10,
                              ckpt_every=20):
        """Real2Sim-style gradient descent (dm_fit_natural_curvature): returns the fitted
        concatenated natural curvature and the loss of every evaluated iterate (host arrays)."""
        tgt = _f64(target_tips)
        if tgt.size != int(nsteps) * self.num_rods * 3:
            raise ValueError(f"target_tips must hold nsteps x n_rods x 3 = {int(nsteps) * self.num_rods * 3} values")
        kb = np.zeros(self.kbar_size) if kbar0 is None else _f64(kbar0).copy()
        if kb.size != self.kbar_size:
            raise ValueError(f"kbar0 must hold {self.kbar_size} values")
        losses = np.zeros(max_iter + 1)
        n = ctypes.c_int(0)
        _check(lib().dm_fit_natural_curvature(self._h, float(dt), int(nsteps), int(ckpt_every), tgt.ctypes.data, 0,
                                              float(alpha0), float(tol), int(max_iter), kb.ctypes.data, 0,
                                              losses.ctypes.data_as(_DP), ctypes.byref(n)),
               "dm_fit_natural_curvature")
        return kb, losses[:n.value]

    @property
    def time(self):
        return lib().dm_time(self._h)

    @property
    def last_kernel_ms(self):
        """Duration of the last step() kernel from HIP events on the simulation's stream."""
        return lib().dm_last_kernel_ms(self._h)

    @property
    def block_size(self):
        return lib().dm_block_size(self._h)


class Mlp:
    """The warm-start network (dm_mlp): float32 master weights, bfloat16 matrix-core kernels."""

    def __init__(self, max_rows, device=0, stream=None):
        if lib().dm_mlp_num_inputs() != NET_IN:
            raise DmError(f"libdmrod.so takes {lib().dm_mlp_num_inputs()} features per row, the binding {NET_IN}: "
                          "rebuild the library")
        h = c_void_p()
        _check(lib().dm_mlp_create(device, stream, int(max_rows), ctypes.byref(h)), "dm_mlp_create")
        self._h = h
        self.max_rows = int(max_rows)
        self.stream = stream

    @staticmethod
    def num_params():
        return lib().dm_mlp_num_params()

    def close(self):
        if getattr(self, "_h", None):
            lib().dm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        if _is_cuda_tensor(params):
            _check(lib().dm_mlp_set_params(self._h, params.data_ptr(), 1), "dm_mlp_set_params")
        else:
            p = np.ascontiguousarray(params, dtype=np.float32)
            _check(lib().dm_mlp_set_params(self._h, p.ctypes.data, 0), "dm_mlp_set_params")

    def get_params(self):
        p = np.zeros(self.num_params(), dtype=np.float32)
        _check(lib().dm_mlp_get_params(self._h, p.ctypes.data, 0), "dm_mlp_get_params")
        return p

    def set_normalisation(self, mean, std, scale):
        m, sd, sc = _sized(mean, NET_IN, "mean"), _sized(std, NET_IN, "std"), _sized(scale, 3, "scale")
        _check(lib().dm_mlp_set_normalisation(self._h, _dp(m), _dp(sd), _dp(sc)), "dm_mlp_set_normalisation")

    def get_normalisation(self):
        m, sd, sc = np.zeros(NET_IN), np.zeros(NET_IN), np.zeros(3)
        _check(lib().dm_mlp_get_normalisation(self._h, _dp(m), _dp(sd), _dp(sc)), "dm_mlp_get_normalisation")
        return m, sd, sc

    def fit_normalisation(self, F, T):
        _check(lib().dm_mlp_fit_normalisation(self._h, F.data_ptr(), T.data_ptr(), F.shape[0]), "dm_mlp_fit_normalisation")

    def forward_noalloc(self, F, out):
        """forward() through dm_mlp_forward_noalloc (static activations, at most
        DM_MLP_NOALLOC_MAX_ROWS rows)."""
        _check(lib().dm_mlp_forward_noalloc(self._h, F.data_ptr(), F.shape[0], out.data_ptr()),
               "dm_mlp_forward_noalloc")
        return out

    def forward(self, F, out):
        _check(lib().dm_mlp_forward(self._h, F.data_ptr(), F.shape[0], out.data_ptr()), "dm_mlp_forward")
        return out

    def gradients(self, F, T, out):
        loss = c_double()
        _check(lib().dm_mlp_gradients(self._h, F.data_ptr(), T.data_ptr(), F.shape[0], out.data_ptr(),
                                      ctypes.byref(loss)), "dm_mlp_gradients")
        return loss.value

    def train_step(self, F, T, lr=1e-3, want_loss=True):
        """One Adam step; returns the batch loss, or None without waiting for the stream when
        want_loss is False."""
        loss = c_double()
        _check(lib().dm_mlp_train_step(self._h, F.data_ptr(), T.data_ptr(), F.shape[0], lr,
                                       ctypes.byref(loss) if want_loss else None), "dm_mlp_train_step")
        return loss.value if want_loss else None

    def train_epoch(self, F, T, perm, batch, lr=1e-3):
        """Adam over the mini-batches perm[0:batch], perm[batch:2 batch], ... of device features
        F [n, NET_IN] and targets T [n, 3] (float64); perm is a device int32 [n].  Returns the mean
        batch loss."""
        import torch
        n = F.shape[0]
        if (F.dtype != torch.float64 or T.dtype != torch.float64 or perm.dtype != torch.int32
                or tuple(F.shape) != (n, NET_IN) or tuple(T.shape) != (n, 3) or tuple(perm.shape) != (n,)
                or not (F.is_contiguous() and T.is_contiguous() and perm.is_contiguous())):
            raise ValueError(f"train_epoch: F [n, {NET_IN}] and T [n, 3] float64, perm [n] int32, contiguous")
        loss = c_double()
        _check(lib().dm_mlp_train_epoch(self._h, F.data_ptr(), T.data_ptr(), perm.data_ptr(), n, int(batch), lr,
                                        ctypes.byref(loss)), "dm_mlp_train_epoch")
        return loss.value


class Contact:
    """Edge-edge contact (dm_contact_*): pair detection inside groups of edges and each pair's
    energy k_c E_c(D) (Eq. 10), gradient, Hessian and friction (Eq. 12-13).  Positions are
    float64 device tensors (n_nodes, 3); outputs are device tensors in the library's layouts."""

    def __init__(self, n_nodes, edges, rod, arc0, ebar, radius, group_start, delta, pair_capacity,
                 device=0, stream=None):
        e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        ne = e.shape[0]
        r = np.ascontiguousarray(rod, dtype=np.int32).reshape(ne)
        a0, eb, rad = (_f64(v, (ne,)) for v in (arc0, ebar, radius))
        gs = np.ascontiguousarray(group_start, dtype=np.int32)
        h = c_void_p()
        _check(lib().dm_contact_create(int(device), stream, int(n_nodes), ne, e.ctypes.data_as(_IP),
                                       r.ctypes.data_as(_IP), _dp(a0), _dp(eb), _dp(rad), int(gs.size - 1),
                                       gs.ctypes.data_as(_IP), float(delta), int(pair_capacity), ctypes.byref(h)),
               "dm_contact_create")
        self._h = h
        self.n_nodes, self.n_edges, self.n_groups, self.cap = int(n_nodes), ne, int(gs.size - 1), int(pair_capacity)
        self.device = device

    @staticmethod
    def from_rods(rods, groups, delta, pair_capacity, device=0, stream=None):
        """rods: [(x0 (N, 3), radius), ...] numbered rod after rod (nodes and edges in order);
        groups: the number of rods in each group, in order.  Rest lengths and arclengths come
        from x0."""
        edges, rod, arc0, ebar, radius, gstart = [], [], [], [], [], [0]
        off, k = 0, 0
        for gsize in groups:
            for _ in range(gsize):
                x0, h = rods[k]
                x0 = np.asarray(x0, dtype=np.float64)
                eb = np.linalg.norm(np.diff(x0, axis=0), axis=1)
                a = np.concatenate([[0.0], np.cumsum(eb)[:-1]])
                for j in range(x0.shape[0] - 1):
                    edges.append((off + j, off + j + 1))
                    rod.append(k)
                    arc0.append(a[j])
                    ebar.append(eb[j])
                    radius.append(h)
                off += x0.shape[0]
                k += 1
            gstart.append(len(edges))
        return Contact(off, edges, rod, arc0, ebar, radius, gstart, delta, pair_capacity, device, stream)

    def close(self):
        if getattr(self, "_h", None):
            lib().dm_contact_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _x(self, x):
        import torch
        if not (x.is_cuda and x.dtype == torch.float64 and x.is_contiguous() and tuple(x.shape) == (self.n_nodes, 3)):
            raise ValueError(f"positions: contiguous float64 device tensor ({self.n_nodes}, 3)")
        return x

    def find(self, x):
        """Pairs at positions x: (pairs [G, cap, 2] int32, dst [G, cap, 3] = D, s, t,
        counts [G] int32, total).  Raises DmError when a group exceeds the capacity."""
        import torch
        x = self._x(x)
        G, cap = self.n_groups, self.cap
        pairs = torch.zeros((G, cap, 2), dtype=torch.int32, device=x.device)
        dst = torch.zeros((G, cap, 3), dtype=torch.float64, device=x.device)
        counts = torch.zeros((G,), dtype=torch.int32, device=x.device)
        tot = c_int()
        _check(lib().dm_contact_find(self._h, x.data_ptr(), pairs.data_ptr(), dst.data_ptr(), counts.data_ptr(),
                                     ctypes.byref(tot)), "dm_contact_find")
        return pairs, dst, counts, tot.value

    def terms(self, x, pairs, counts, k_c, x_prev=None, dt=0.0, mu=0.0, nu=1.0, hessian=True, friction=False):
        """Per pair slot: energy [G, cap], gradient [G, 12, cap], Hessian [G, 144, cap] (or
        None), friction forces [G, 12, cap] (or None; needs x_prev, dt, mu, nu)."""
        import torch
        x = self._x(x)
        G, cap = self.n_groups, self.cap
        z = dict(dtype=torch.float64, device=x.device)
        energy = torch.zeros((G, cap), **z)
        grad = torch.zeros((G, 12, cap), **z)
        hess = torch.zeros((G, 144, cap), **z) if hessian else None
        fric = torch.zeros((G, 12, cap), **z) if friction else None
        xp = self._x(x_prev).data_ptr() if x_prev is not None else None
        _check(lib().dm_contact_terms(self._h, x.data_ptr(), xp, float(dt), float(k_c), float(mu), float(nu),
                                      pairs.data_ptr(), counts.data_ptr(), energy.data_ptr(), grad.data_ptr(),
                                      hess.data_ptr() if hess is not None else None,
                                      fric.data_ptr() if fric is not None else None), "dm_contact_terms")
        return energy, grad, hess, fric

    @property
    def last_find_ms(self):
        return lib().dm_contact_last_ms(self._h, 0)

    @property
    def last_terms_ms(self):
        return lib().dm_contact_last_ms(self._h, 1)


def _is_cuda_tensor(a):
    return getattr(a, "is_cuda", False) and hasattr(a, "data_ptr")


def tip_trajectory(kbar, sim, start, dt, nsteps, ckpt_every=20):
    """Differentiable GPU rollout: the tip trajectory (nsteps, n_rods, 3) of `sim` started from
    the checkpoint `start` (checkpoint_torch) with natural curvature `kbar` (concatenated,
    float64 device tensor).  Its backward is the library's discrete adjoint (dm_adjoint).
    The Sim should run on torch's current stream."""
    import torch

    class _TipTrajectory(torch.autograd.Function):
        @staticmethod
        def forward(ctx, k):
            sim.restore(start)
            sim.set_natural_curvature_all(k)
            tips = torch.empty((nsteps, sim.num_rods, 3), dtype=torch.float64, device=k.device)
            sim.rollout(dt, nsteps, ckpt_every, out=tips)
            return tips

        @staticmethod
        def backward(ctx, g):
            grad = torch.empty(sim.kbar_size, dtype=torch.float64, device=g.device)
            sim.adjoint(g.contiguous(), out=grad)
            return grad

    return _TipTrajectory.apply(kbar)


def sim_from_description(desc, **overrides):
    """Build and finalize a Sim from a `workloads` description (marshalling only)."""
    kw = dict(gravity=desc["gravity"], newton_tol=desc["tol"], max_iter=desc["max_iter"],
              floor=desc.get("floor"), damping=desc.get("damping", 0.0),
              line_search=desc.get("line_search", False))
    kw.update(overrides)
    sim = Sim(**kw)
    for r in desc["rods"]:
        rid = sim.add_rod(r["x0"], r["radius"], r["E"], r["poisson"], r["density"])
        if r["fixed_nodes"]:
            sim.fix_nodes(rid, r["fixed_nodes"])
        if r["fixed_edges"]:
            sim.fix_edges(rid, r["fixed_edges"])
        if r.get("kbar") is not None:
            sim.set_natural_curvature(rid, r["kbar"])
        if r.get("actuation") is not None:
            sim.set_actuation_sine(rid, *r["actuation"])
        if r.get("force") is not None or r.get("moment") is not None:
            sim.set_external_load(rid, r.get("force"), r.get("moment"))
    for (ra, na, rb, nb) in desc["joints"]:
        sim.add_joint(ra, na, rb, nb)
    sim.finalize()
    if desc.get("self_contact"):
        sc = desc["self_contact"]
        sim.set_self_contact(sc["delta"], sc["k_c"], sc.get("mu", 0.0), sc.get("nu", 1e-3))
    if "initial_tip_velocity" in desc:
        for rid in range(len(desc["rods"])):
            x, th, v, om = sim.rod_state(rid)
            v[-1] = desc["initial_tip_velocity"]
            sim.set_rod_state(rid, v=v)
    return sim
