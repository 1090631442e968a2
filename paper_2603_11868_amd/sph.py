"""ctypes binding of libsph (include/sph.h).

The functions below carry the names of the C ABI and only marshal arguments:
every stage runs in the HIP kernels of libsph.  PyTorch provides the device
memory (``torch.empty(..., device="cuda")``) and the stream
(``torch.cuda.current_stream().cuda_stream``).  The library must be built
(``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK = 0
SPH_FP64 = 0
SPH_MIXED = 1
SPH_NDIAG = 16
SPH_FLAG_CLAMPED = 1
SPH_FLAG_NONFINITE = 2
SPH_FLAG_CAPACITY = 4

STATUS_NAMES = {0: "SPH_OK", -1: "SPH_E_ARG", -2: "SPH_E_STATE", -3: "SPH_E_HIP",
                -4: "SPH_E_CAPACITY", -5: "SPH_E_UNSUPPORTED"}

DIAG_NAMES = ("vmax", "amax", "mass", "mom_x", "mom_y", "mom_z", "kinetic",
              "potential", "internal", "ff_residual", "rho_mean_dev", "clamped",
              "pairs", "ff_impulse", "time", "steps")

# exported symbols declared in include/sph.h
SYMBOLS = ("sph_last_error", "sph_create", "sph_destroy", "sph_get_info", "sph_get_grid",
           "sph_workspace_size", "sph_bind", "sph_prime", "sph_build_cells", "sph_sort",
           "sph_density", "sph_forces", "sph_integrate", "sph_step_batched",
           "sph_poll_errors", "sph_set_timing", "sph_stage_times", "sph_stage_name",
           "sph_stage_count", "sph_substeps", "sph_cell_builds", "sph_set_timing_mask",
           "sph_bind_static")
SPH_STATIC_SCRATCH_BYTES = 32 << 20

SPH_SCHEME_WCSPH, SPH_SCHEME_DUAL = 0, 1
SPH_KEYS_ROW_MAJOR, SPH_KEYS_MORTON_TILES = 0, 1
SPH_POLICY_DEVICE, SPH_POLICY_HOST = 0, 1
# parameters of the dual-criteria scheme as published (advection and acoustic
# Courant numbers, dissipation limiter slope)
DUAL_CFL_ADV, DUAL_CFL_AC, DUAL_ETA = 0.25, 0.6, 3.0


class SphError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class sph_instance_desc(C.Structure):
    _fields_ = [("n_fluid", C.c_int32), ("n_wall", C.c_int32),
                ("tank_lo", C.c_double * 3), ("tank_hi", C.c_double * 3), ("c0", C.c_double)]


class sph_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("n_instances", C.c_int32),
                ("reorder_every", C.c_int32), ("dx", C.c_double), ("h", C.c_double),
                ("rho0", C.c_double), ("alpha", C.c_double), ("eps", C.c_double),
                ("cfl_ac", C.c_double), ("cfl_f", C.c_double), ("g", C.c_double * 3),
                ("inst", C.POINTER(sph_instance_desc)), ("block_threads", C.c_int32),
                ("use_graph", C.c_int32), ("list_cap", C.c_int32),
                ("prefetch", C.c_int32), ("scheme", C.c_int32), ("key_order", C.c_int32),
                ("cfl_adv", C.c_double), ("eta", C.c_double), ("skin", C.c_double),
                ("build", C.c_int32), ("policy", C.c_int32)]


class sph_buffers(C.Structure):
    _fields_ = [("x", C.c_void_p), ("v", C.c_void_p), ("a", C.c_void_p), ("rho", C.c_void_p),
                ("id", C.c_void_p), ("key", C.c_void_p), ("perm", C.c_void_p),
                ("count", C.c_void_p), ("xw", C.c_void_p), ("wall_perm", C.c_void_p),
                ("cell_start", C.c_void_p), ("wall_start", C.c_void_p), ("dt", C.c_void_p),
                ("diag", C.c_void_p), ("workspace", C.c_void_p)]


class sph_info(C.Structure):
    _fields_ = [("n_fluid", C.c_int64), ("n_wall", C.c_int64), ("n_cells", C.c_int64),
                ("workspace_bytes", C.c_size_t), ("sigma0", C.c_double), ("mass", C.c_double),
                ("cell_size", C.c_double), ("steps_done", C.c_int64), ("substeps_done", C.c_int64)]


_lib = None


def lib():
    """Load libsph.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(hipcc for gfx950) before using the HIP path")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.sph_last_error.restype = C.c_char_p
        L.sph_create.argtypes = [C.POINTER(sph_params), C.POINTER(vp)]
        L.sph_destroy.argtypes = [vp]
        L.sph_destroy.restype = None
        L.sph_get_info.argtypes = [vp, C.POINTER(sph_info)]
        L.sph_get_grid.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32)]
        L.sph_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.sph_bind.argtypes = [vp, C.POINTER(sph_buffers), vp]
        L.sph_bind_static.argtypes = [vp, C.POINTER(sph_buffers), vp]
        for n in ("sph_prime", "sph_build_cells", "sph_density", "sph_forces"):
            getattr(L, n).argtypes = [vp, vp]
        L.sph_sort.argtypes = [vp, C.c_int32, vp]
        L.sph_integrate.argtypes = [vp, C.c_int32, vp]
        L.sph_step_batched.argtypes = [vp, C.c_int32, vp]
        L.sph_substeps.argtypes = [vp, C.POINTER(C.c_int32), vp]
        L.sph_cell_builds.argtypes = [vp, C.POINTER(C.c_int64), vp]
        L.sph_poll_errors.argtypes = [vp, C.POINTER(C.c_uint32), vp]
        L.sph_set_timing.argtypes = [vp, C.c_int32]
        L.sph_set_timing_mask.argtypes = [vp, C.c_uint32]
        L.sph_stage_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32,
                                      C.c_int32, vp]
        L.sph_stage_name.argtypes = [C.c_int32]
        L.sph_stage_name.restype = C.c_char_p
        L.sph_stage_count.restype = C.c_int32
        for n in SYMBOLS:
            f = getattr(L, n)
            if n not in ("sph_last_error", "sph_destroy", "sph_stage_name", "sph_stage_count"):
                f.restype = C.c_int
        _lib = L
    return _lib


def _check(status):
    if status != SPH_OK:
        raise SphError(status, lib().sph_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ---- the C ABI, one function per entry point -----------------------------

def sph_last_error():
    return lib().sph_last_error().decode()


def sph_create(params: sph_params):
    ctx = C.c_void_p()
    _check(lib().sph_create(C.byref(params), C.byref(ctx)))
    return ctx


def sph_destroy(ctx):
    lib().sph_destroy(ctx)


def sph_get_info(ctx) -> sph_info:
    info = sph_info()
    _check(lib().sph_get_info(ctx, C.byref(info)))
    return info


def sph_get_grid(ctx, b):
    lo = (C.c_double * 3)()
    nc = (C.c_int32 * 3)()
    base = C.c_int32()
    _check(lib().sph_get_grid(ctx, int(b), lo, nc, C.byref(base)))
    return tuple(lo), tuple(nc), int(base.value)


def sph_workspace_size(ctx) -> int:
    n = C.c_size_t()
    _check(lib().sph_workspace_size(ctx, C.byref(n)))
    return int(n.value)


def sph_bind(ctx, buffers: sph_buffers, stream=None):
    _check(lib().sph_bind(ctx, C.byref(buffers), _stream(stream)))


def sph_bind_static(ctx, buffers: sph_buffers, stream=None):
    _check(lib().sph_bind_static(ctx, C.byref(buffers), _stream(stream)))


def sph_prime(ctx, stream=None):
    _check(lib().sph_prime(ctx, _stream(stream)))


def sph_build_cells(ctx, stream=None):
    _check(lib().sph_build_cells(ctx, _stream(stream)))


def sph_sort(ctx, reorder=0, stream=None):
    _check(lib().sph_sort(ctx, int(reorder), _stream(stream)))


def sph_density(ctx, stream=None):
    _check(lib().sph_density(ctx, _stream(stream)))


def sph_forces(ctx, stream=None):
    _check(lib().sph_forces(ctx, _stream(stream)))


def sph_integrate(ctx, half, stream=None):
    _check(lib().sph_integrate(ctx, int(half), _stream(stream)))


def sph_step_batched(ctx, n_steps, stream=None):
    _check(lib().sph_step_batched(ctx, int(n_steps), _stream(stream)))


def sph_substeps(ctx, n_instances, stream=None):
    out = (C.c_int32 * n_instances)()
    _check(lib().sph_substeps(ctx, out, _stream(stream)))
    return [int(v) for v in out]


def sph_cell_builds(ctx, stream=None) -> int:
    n = C.c_int64()
    _check(lib().sph_cell_builds(ctx, C.byref(n), _stream(stream)))
    return int(n.value)


def sph_poll_errors(ctx, stream=None) -> int:
    f = C.c_uint32()
    _check(lib().sph_poll_errors(ctx, C.byref(f), _stream(stream)))
    return int(f.value)


def sph_set_timing(ctx, enable):
    _check(lib().sph_set_timing(ctx, int(bool(enable))))


def sph_set_timing_mask(ctx, mask):
    _check(lib().sph_set_timing_mask(ctx, int(mask)))


def sph_stage_count() -> int:
    return int(lib().sph_stage_count())


def sph_stage_name(i) -> str:
    return lib().sph_stage_name(int(i)).decode()


def sph_stage_times(ctx, reset=True, stream=None):
    n = sph_stage_count()
    ms = (C.c_double * n)()
    cnt = (C.c_int64 * n)()
    _check(lib().sph_stage_times(ctx, ms, cnt, n, int(bool(reset)), _stream(stream)))
    return {sph_stage_name(i): (ms[i], int(cnt[i])) for i in range(n)}


# ---- convenience: a bound simulation over torch device buffers -----------

class Simulation:
    """Device buffers (torch) for a ``dambreak.Case`` bound to a libsph context.

    Storage arrays are component-major: ``x[a, i]``.  Particle ids are global:
    instance b owns ids fluid_offset[b] .. fluid_offset[b] + n_b - 1.
    """

    def __init__(self, case, precision="fp64", reorder_every=None, block_threads=0,
                 use_graph=False, device="cuda", alpha=None, g=None,
                 cfl=None, velocities=None, densities=None, list_cap=0, prefetch=0,
                 scheme="wcsph", skin=0.0, key_order="row", static_scratch=False, build=None,
                 tuned=False, policy="device"):
        """policy: "device" (the HIP kernels; buffers in GPU memory) or "host"
        (the same step bodies on the host's threads; buffers in host memory,
        FP64 only).  The host policy is used only when asked for."""
        import torch
        self.torch = torch
        self.case = case
        self.tuned = None
        if tuned:
            # launch parameters from the autotuner's cache for this workload
            # (block size, list build, candidate prefetch), where present
            from . import tune as _tune
            best = _tune.lookup(case, precision)
            if best:
                # only the parameters the caller left unset
                self.tuned = {k: best[k] for k in ("block_threads", "build", "prefetch") if k in best}
                if not block_threads:
                    block_threads = self.tuned.get("block_threads", 0)
                if build is None:
                    build = self.tuned.get("build", 0)
                if not prefetch:
                    prefetch = self.tuned.get("prefetch", 0)
        if build is None:
            build = 0
        if policy not in ("device", "host"):
            raise ValueError(f"unknown policy {policy!r}")
        self.policy = policy
        # host contexts take no stream (calls with None would ask torch for
        # the current GPU stream)
        self._s = 0 if policy == "host" else None
        if policy == "host":
            device = "cpu"
        self.dim = dim = case.dim
        self.device = torch.device(device)
        B = len(case.instances)
        descs = (sph_instance_desc * B)()
        for b, inst in enumerate(case.instances):
            d = descs[b]
            d.n_fluid = inst.n_fluid
            d.n_wall = inst.n_wall
            for a in range(3):
                d.tank_lo[a] = float(inst.tank_lo[a])
                d.tank_hi[a] = float(inst.tank_hi[a])
            d.c0 = float(inst.c0)
        p = sph_params()
        p.dim = dim
        p.precision = SPH_MIXED if precision == "mixed" else SPH_FP64
        p.n_instances = B
        p.reorder_every = case.reorder_every if reorder_every is None else int(reorder_every)
        p.dx, p.h, p.rho0 = case.dx, case.h, case.rho0
        p.alpha = case.alpha if alpha is None else float(alpha)
        p.eps = case.eps
        p.cfl_ac = case.cfl_ac if cfl is None else float(cfl)
        p.cfl_f = case.cfl_f if cfl is None else float(cfl)
        gv = case.g if g is None else np.asarray(list(g) + [0.0] * (3 - len(g)), dtype=float)
        for a in range(3):
            p.g[a] = float(gv[a])
        p.inst = descs
        p.block_threads = int(block_threads)
        p.use_graph = int(bool(use_graph))
        p.list_cap = int(list_cap)
        p.prefetch = int(prefetch)
        p.build = int(build)
        p.skin = float(skin)               # Verlet skin, a length (0: none)
        p.key_order = {"row": SPH_KEYS_ROW_MAJOR, "morton": SPH_KEYS_MORTON_TILES}[key_order]
        p.policy = SPH_POLICY_HOST if policy == "host" else SPH_POLICY_DEVICE
        if scheme == "dual":
            p.scheme = SPH_SCHEME_DUAL
            p.cfl_ac = DUAL_CFL_AC if cfl is None else float(cfl)
            p.cfl_adv, p.eta = DUAL_CFL_ADV, DUAL_ETA
        elif scheme != "wcsph":
            raise ValueError(f"unknown scheme {scheme!r}")
        self.scheme = scheme
        self._descs = descs
        self.params = p
        self.precision = precision
        self.ctx = sph_create(p)
        info = sph_get_info(self.ctx)
        self.info = info
        N, Nw, Cn = int(info.n_fluid), int(info.n_wall), int(info.n_cells)
        self.N, self.Nw, self.C, self.B = N, Nw, Cn, B
        self.fluid_offset = np.concatenate([[0], np.cumsum([i.n_fluid for i in case.instances])])
        self.wall_offset = np.concatenate([[0], np.cumsum([i.n_wall for i in case.instances])])
        dev = self.device
        f64, i32 = torch.float64, torch.int32
        xs = np.concatenate([i.fluid[:, :dim] for i in case.instances], 0) if N else np.zeros((0, dim))
        ws = np.concatenate([i.wall[:, :dim] for i in case.instances], 0) if Nw else np.zeros((0, dim))
        self.x = torch.from_numpy(np.ascontiguousarray(xs.T)).to(dev)
        if velocities is None:
            self.v = torch.zeros((dim, N), dtype=f64, device=dev)
        else:
            self.v = torch.from_numpy(np.ascontiguousarray(np.asarray(velocities, float).T)).to(dev)
        self.a = torch.zeros((dim, N), dtype=f64, device=dev)
        if densities is None:
            self.rho = torch.full((N,), case.rho0, dtype=f64, device=dev)
        else:
            self.rho = torch.from_numpy(np.asarray(densities, float).copy()).to(dev)
        self.id = torch.arange(N, dtype=i32, device=dev)
        self.key = torch.zeros(N, dtype=i32, device=dev)
        self.perm = torch.zeros(N, dtype=i32, device=dev)
        self.count = torch.zeros(N, dtype=i32, device=dev)
        self.xw = torch.from_numpy(np.ascontiguousarray(ws.T)).to(dev)
        self.wall_perm = torch.zeros(max(Nw, 1), dtype=i32, device=dev)
        self.cell_start = torch.zeros(Cn + 1, dtype=i32, device=dev)
        self.wall_start = torch.zeros(Cn + 1, dtype=i32, device=dev)
        self.dt = torch.zeros(B, dtype=f64, device=dev)
        self.diag = torch.zeros((B, SPH_NDIAG), dtype=f64, device=dev)
        if static_scratch or policy == "host":
            # the library's own workspace (sph_bind_static), or none (the host
            # policy keeps its scratch itself): nothing allocated here
            self.workspace = None
            wptr = 0
        else:
            self.workspace = torch.empty(int(info.workspace_bytes) + 256, dtype=torch.uint8, device=dev)
            wptr = self.workspace.data_ptr()
            wptr = (wptr + 255) & ~255
        bufs = sph_buffers()
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t.numel() else C.c_void_p(0)
        bufs.x, bufs.v, bufs.a, bufs.rho = ptr(self.x), ptr(self.v), ptr(self.a), ptr(self.rho)
        bufs.id, bufs.key, bufs.perm, bufs.count = ptr(self.id), ptr(self.key), ptr(self.perm), ptr(self.count)
        bufs.xw, bufs.wall_perm = ptr(self.xw), ptr(self.wall_perm)
        bufs.cell_start, bufs.wall_start = ptr(self.cell_start), ptr(self.wall_start)
        bufs.dt, bufs.diag = ptr(self.dt), ptr(self.diag)
        bufs.workspace = C.c_void_p(wptr)
        self.buffers = bufs
        if static_scratch:
            sph_bind_static(self.ctx, bufs)
        else:
            sph_bind(self.ctx, bufs, stream=self._s)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            sph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stages --------------------------------------------------------------
    def prime(self):
        sph_prime(self.ctx, stream=self._s)

    def step(self, n=1):
        sph_step_batched(self.ctx, n, stream=self._s)

    def build_cells(self):
        sph_build_cells(self.ctx, stream=self._s)

    def sort(self, reorder=False):
        sph_sort(self.ctx, int(reorder), stream=self._s)

    def density(self):
        sph_density(self.ctx, stream=self._s)

    def forces(self):
        sph_forces(self.ctx, stream=self._s)

    def integrate(self, half):
        sph_integrate(self.ctx, half, stream=self._s)

    def poll_errors(self):
        return sph_poll_errors(self.ctx, stream=self._s)

    def grid(self, b=0):
        return sph_get_grid(self.ctx, b)

    @property
    def steps_done(self):
        return int(sph_get_info(self.ctx).steps_done)

    def cell_builds(self):
        return sph_cell_builds(self.ctx, stream=self._s)

    def synchronize(self):
        if self.policy == "device":
            self.torch.cuda.synchronize(self.device)

    # -- host copies ---------------------------------------------------------
    def host(self):
        """Host copies of the state (storage order), after a synchronise."""
        self.synchronize()
        t = lambda x: x.detach().cpu().numpy()
        return {
            "x": t(self.x).T.copy(), "v": t(self.v).T.copy(), "a": t(self.a).T.copy(),
            "rho": t(self.rho), "id": t(self.id), "key": t(self.key), "perm": t(self.perm),
            "count": t(self.count), "cell_start": t(self.cell_start),
            "wall_start": t(self.wall_start), "wall_perm": t(self.wall_perm)[:self.Nw],
            "dt": t(self.dt), "diag": t(self.diag),
        }

    def by_id(self, arr, ids):
        out = np.empty_like(arr)
        out[ids] = arr
        return out
