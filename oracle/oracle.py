"""Python front end of the plain FP64 CPU reference (``sph_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the CPU baseline
leg of the benchmark may import this module; the product package never does.
It shares no code with the HIP library: the C source here is compiled with gcc
on its own and loaded through ctypes.

State is held in numpy arrays (storage order, ``dim`` doubles per particle).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NDIAG = 16

DIAG_NAMES = ("vmax", "amax", "mass", "mom_x", "mom_y", "mom_z", "kinetic",
              "potential", "internal", "ff_residual", "rho_mean_dev", "clamped",
              "pairs", "ff_impulse", "time", "steps")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("dx", C.c_double), ("h", C.c_double),
        ("rho0", C.c_double), ("c0", C.c_double), ("alpha", C.c_double),
        ("eps", C.c_double), ("cfl_ac", C.c_double), ("cfl_f", C.c_double),
        ("g", C.c_double * 3), ("tank_lo", C.c_double * 3), ("tank_hi", C.c_double * 3),
        ("reorder_every", C.c_int),
        ("cs", C.c_double), ("inv_cs", C.c_double), ("cut2", C.c_double),
        ("sigma0", C.c_double), ("mass", C.c_double), ("lo", C.c_double * 3),
        ("ncell", C.c_int * 3), ("ncells", C.c_int),
    ]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _State(C.Structure):
    _fields_ = [
        ("n", C.c_int), ("nw", C.c_int),
        ("x", _dp), ("v", _dp), ("a", _dp), ("rho", _dp), ("P", _dp),
        ("id", _ip), ("key", _ip), ("perm", _ip), ("count", _ip), ("start", _ip),
        ("xw", _dp), ("wkey", _ip), ("wperm", _ip), ("wstart", _ip),
        ("dt", _dp), ("diag", _dp), ("step", C.POINTER(C.c_int64)),
    ]


class _Dual(C.Structure):
    _fields_ = [("cfl_adv", C.c_double), ("cfl_ac", C.c_double), ("eta", C.c_double)]


class _DualState(C.Structure):
    _fields_ = [("x_adv", _dp), ("drho", _dp), ("pres", _dp), ("a_ff", _dp),
                ("Dt", C.c_double), ("dt", C.c_double), ("nsub", C.c_int)]


# parameters of the dual-criteria scheme
DUAL_CFL_ADV = 0.25
DUAL_CFL_AC = 0.6
DUAL_ETA = 3.0

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        L.or_kernel_alpha.restype = C.c_double
        L.or_kernel_alpha.argtypes = [C.c_int, C.c_double]
        L.or_W.restype = C.c_double
        L.or_W.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_F.restype = C.c_double
        L.or_F.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_sigma0.restype = C.c_double
        L.or_sigma0.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_setup.restype = C.c_int
        L.or_setup.argtypes = [C.POINTER(_Params)]
        L.or_keys.restype = C.c_int
        L.or_keys.argtypes = [C.POINTER(_Params), C.c_int, _dp, _ip]
        L.or_sort.restype = None
        L.or_sort.argtypes = [C.c_int, _ip, C.c_int, _ip, _ip]
        ps = [C.POINTER(_Params), C.POINTER(_State)]
        for name, extra in (("or_reorder", []), ("or_density", [C.c_double]),
                            ("or_forces", [_dp]), ("or_half1", [C.c_double]),
                            ("or_half2", [C.c_double]),
                            ("or_reduce", [_dp, C.c_int, C.c_double])):
            f = getattr(L, name)
            f.restype = None
            f.argtypes = ps + extra
        for name in ("or_bind_walls", "or_prime"):
            f = getattr(L, name)
            f.restype = C.c_int
            f.argtypes = ps
        L.or_step.restype = C.c_int
        L.or_step.argtypes = ps + [C.c_int]
        L.or_num_threads.restype = C.c_int
        L.or_num_threads.argtypes = []
        L.or_riemann.restype = None
        L.or_riemann.argtypes = [C.c_double] * 8 + [_dp, _dp]
        pd = [C.POINTER(_Params), C.POINTER(_Dual), C.POINTER(_State), C.POINTER(_DualState)]
        L.or_dual_plan.restype = None
        L.or_dual_plan.argtypes = pd
        L.or_dual_summation.restype = None
        L.or_dual_summation.argtypes = [pd[0], pd[2], pd[3]]
        L.or_dual_first_half.restype = None
        L.or_dual_first_half.argtypes = [pd[0], pd[2], pd[3], C.c_double]
        L.or_dual_pressure.restype = None
        L.or_dual_pressure.argtypes = pd + [C.c_double]
        L.or_dual_second_half.restype = None
        L.or_dual_second_half.argtypes = [pd[0], pd[2], C.c_double]
        L.or_dual_density.restype = None
        L.or_dual_density.argtypes = pd + [C.c_double]
        L.or_dual_prime.restype = C.c_int
        L.or_dual_prime.argtypes = pd
        L.or_dual_step.restype = C.c_int
        L.or_dual_step.argtypes = pd + [C.c_int]
        _lib = L
    return _lib


def num_threads():
    return int(lib().or_num_threads())


def riemann(rho_l, p_l, u_l, rho_r, p_r, u_r, c0, eta=DUAL_ETA):
    """Interface pressure and normal velocity of the acoustic Riemann problem
    between a left and a right state (dissipation limited by eta)."""
    ps, us = C.c_double(), C.c_double()
    lib().or_riemann(float(rho_l), float(p_l), float(u_l), float(rho_r), float(p_r), float(u_r),
                     float(c0), float(eta), C.byref(ps), C.byref(us))
    return ps.value, us.value


def W(dim, h, r):
    return lib().or_W(dim, h, r)


def F(dim, h, r):
    return lib().or_F(dim, h, r)


def kernel_alpha(dim, h):
    return lib().or_kernel_alpha(dim, h)


def sigma0(dim, dx, h):
    return lib().or_sigma0(dim, dx, h)


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


class OracleSim:
    """One independent instance simulated by the FP64 reference.

    ``fluid`` and ``wall`` are (n, dim) float64 position arrays; ``v`` an
    optional initial velocity.  Other keywords override the run parameters.
    """

    def __init__(self, dim, dx, h, tank_lo, tank_hi, fluid, wall, c0,
                 rho0=1000.0, alpha=0.1, eps=0.01, cfl_ac=0.25, cfl_f=0.25,
                 g=None, reorder_every=20, v=None, rho=None):
        L = lib()
        self.dim = dim
        p = _Params()
        p.dim = dim
        p.dx, p.h, p.rho0, p.c0 = dx, h, rho0, c0
        p.alpha, p.eps, p.cfl_ac, p.cfl_f = alpha, eps, cfl_ac, cfl_f
        gv = np.zeros(3)
        if g is None:
            gv[dim - 1] = -9.81
        else:
            gv[:len(g)] = g
        for a in range(3):
            p.g[a] = gv[a]
            p.tank_lo[a] = float(tank_lo[a]) if a < len(tank_lo) else 0.0
            p.tank_hi[a] = float(tank_hi[a]) if a < len(tank_hi) else 0.0
        p.reorder_every = int(reorder_every)
        rc = L.or_setup(C.byref(p))
        if rc != 0:
            raise ValueError(f"oracle setup failed ({rc})")
        self.p = p
        n = int(fluid.shape[0])
        nw = int(wall.shape[0])
        self.n, self.nw = n, nw
        self.x = np.ascontiguousarray(fluid[:, :dim], dtype=np.float64).copy()
        self.v = np.zeros((n, dim)) if v is None else np.ascontiguousarray(v, dtype=np.float64).copy()
        self.a = np.zeros((n, dim))
        self.rho = np.full(n, rho0) if rho is None else np.ascontiguousarray(rho, dtype=np.float64).copy()
        self.P = np.zeros(n)
        self.id = np.arange(n, dtype=np.int32)
        self.key = np.zeros(n, dtype=np.int32)
        self.perm = np.zeros(n, dtype=np.int32)
        self.count = np.zeros(n, dtype=np.int32)
        self.start = np.zeros(p.ncells + 1, dtype=np.int32)
        self.xw = np.ascontiguousarray(wall[:, :dim], dtype=np.float64).copy()
        self.wkey = np.zeros(max(nw, 1), dtype=np.int32)
        self.wperm = np.zeros(max(nw, 1), dtype=np.int32)
        self.wstart = np.zeros(p.ncells + 1, dtype=np.int32)
        self.dt = np.zeros(1)
        self.diag = np.zeros(NDIAG)
        self.stepc = np.zeros(1, dtype=np.int64)
        self.a_ff = np.zeros((max(n, 1), dim))
        s = _State()
        s.n, s.nw = n, nw
        s.x, s.v, s.a, s.rho, s.P = _d(self.x), _d(self.v), _d(self.a), _d(self.rho), _d(self.P)
        s.id, s.key, s.perm, s.count, s.start = _i(self.id), _i(self.key), _i(self.perm), _i(self.count), _i(self.start)
        s.xw, s.wkey, s.wperm, s.wstart = _d(self.xw), _i(self.wkey), _i(self.wperm), _i(self.wstart)
        s.dt, s.diag, s.step = _d(self.dt), _d(self.diag), self.stepc.ctypes.data_as(C.POINTER(C.c_int64))
        self.s = s
        self.wall_clamped = L.or_bind_walls(C.byref(p), C.byref(s))

    @classmethod
    def from_case(cls, case, index=0, **kw):
        inst = case.instances[index]
        args = dict(rho0=case.rho0, alpha=case.alpha, eps=case.eps, cfl_ac=case.cfl_ac,
                    cfl_f=case.cfl_f, g=case.g[:case.dim], reorder_every=case.reorder_every)
        args.update(kw)
        return cls(case.dim, case.dx, case.h, inst.tank_lo, inst.tank_hi, inst.fluid,
                   inst.wall, inst.c0, **args)

    # -- derived constants ------------------------------------------------
    @property
    def sigma0(self):
        return self.p.sigma0

    @property
    def mass(self):
        return self.p.mass

    @property
    def ncells(self):
        return self.p.ncells

    @property
    def ncell(self):
        return tuple(self.p.ncell[a] for a in range(3))

    @property
    def lo(self):
        return tuple(self.p.lo[a] for a in range(3))

    @property
    def step_count(self):
        return int(self.stepc[0])

    # -- stages ------------------------------------------------------------
    def keys(self):
        return lib().or_keys(C.byref(self.p), self.n, _d(self.x), _i(self.key))

    def sort(self):
        lib().or_sort(self.n, _i(self.key), self.p.ncells, _i(self.perm), _i(self.start))

    def reorder(self):
        lib().or_reorder(C.byref(self.p), C.byref(self.s))

    def density(self, dt):
        lib().or_density(C.byref(self.p), C.byref(self.s), float(dt))

    def forces(self):
        lib().or_forces(C.byref(self.p), C.byref(self.s), _d(self.a_ff))

    def half1(self, dt):
        lib().or_half1(C.byref(self.p), C.byref(self.s), float(dt))

    def half2(self, dt):
        lib().or_half2(C.byref(self.p), C.byref(self.s), float(dt))

    def reduce(self, clamped=0, dt_used=0.0):
        lib().or_reduce(C.byref(self.p), C.byref(self.s), _d(self.a_ff), int(clamped), float(dt_used))

    def prime(self):
        return lib().or_prime(C.byref(self.p), C.byref(self.s))

    def step(self, nsteps=1):
        return lib().or_step(C.byref(self.p), C.byref(self.s), int(nsteps))

    # -- views indexed by particle id -------------------------------------
    # -- second scheme: dual-criteria time stepping ---------------------
    def _dual(self):
        if getattr(self, "_dstate", None) is None:
            n, dim = max(self.n, 1), self.dim
            self.x_adv = np.zeros((n, dim))
            self.drho = np.zeros(n)
            self.pres = np.zeros(n)
            self.a_ff_dual = np.zeros((n, dim))
            ds = _DualState()
            ds.x_adv, ds.drho, ds.pres, ds.a_ff = (_d(self.x_adv), _d(self.drho), _d(self.pres),
                                                   _d(self.a_ff_dual))
            self._dstate = ds
            dp = _Dual()
            dp.cfl_adv, dp.cfl_ac, dp.eta = DUAL_CFL_ADV, DUAL_CFL_AC, DUAL_ETA
            self._dparams = dp
        return self._dparams, self._dstate

    def dual_prime(self):
        dp, ds = self._dual()
        return lib().or_dual_prime(C.byref(self.p), C.byref(dp), C.byref(self.s), C.byref(ds))

    def dual_step(self, nsteps=1):
        """nsteps advection steps, each with its acoustic sub-steps."""
        dp, ds = self._dual()
        return lib().or_dual_step(C.byref(self.p), C.byref(dp), C.byref(self.s), C.byref(ds), int(nsteps))

    def dual_plan(self):
        """(advection step, sub-steps, sub-step) of the next advection step."""
        dp, ds = self._dual()
        return ds.Dt, ds.nsub, ds.dt

    def dual_stage(self, name, dt=0.0):
        """One stage of the second scheme (summation, first_half, pressure,
        second_half, density), for tests."""
        dp, ds = self._dual()
        L, P, S = lib(), C.byref(self.p), C.byref(self.s)
        if name == "summation":
            L.or_dual_summation(P, S, C.byref(ds))
        elif name == "first_half":
            L.or_dual_first_half(P, S, C.byref(ds), float(dt))
        elif name == "pressure":
            L.or_dual_pressure(P, C.byref(dp), S, C.byref(ds), float(dt))
        elif name == "second_half":
            L.or_dual_second_half(P, S, float(dt))
        elif name == "density":
            L.or_dual_density(P, C.byref(dp), S, C.byref(ds), float(dt))
        else:
            raise ValueError(name)

    def by_id(self, arr):
        out = np.empty_like(arr)
        out[self.id] = arr
        return out

    def sorted_ids(self):
        """Particle ids in sorted (cell) order: id[perm[k]]."""
        return self.id[self.perm]

    def cell_end(self):
        return self.start[1:].copy()
