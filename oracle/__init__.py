"""CPU FP64 oracle of the sG-PM particle method (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product.  Both take the same plain parameter
dictionaries (see ``workloads``), each translating them into its own types.

The C source ``sgpm_oracle.c`` follows Algorithm 2 of the paper (Algorithm 1
when there is no uncertainty) step by step; this module only marshals numpy
arrays through ctypes and computes the expectation/variance over z of the
per-node moments with the nodal quadrature (Sec. 4.2).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgpm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sgpm.so")

Q_E = 1.602176634e-19


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no fast-math, no FP contraction."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("dim_z", C.c_int), ("degree", C.c_int), ("nodes_1d", C.c_int),
        ("n_particles", C.c_long),
        ("gap_mode", C.c_int), ("gap_dim", C.c_int),
        ("gap0", C.c_double), ("gap_rel", C.c_double),
        ("field_dim", C.c_int), ("field0", C.c_double), ("field_rel", C.c_double),
        ("fermi_eV", C.c_double), ("temp_K", C.c_double), ("alpha", C.c_double),
        ("nk", C.c_int), ("lk_eV", C.c_double),
        ("pauli", C.c_int), ("final_state", C.c_int),
        ("rate_scale", C.c_double * 6),
        ("seed", C.c_uint64), ("instance", C.c_uint32), ("c_max", C.c_int),
        ("splitting", C.c_int), ("init_temp_K", C.c_double),
    ]


_lib = None


def lib_path() -> str:
    """The shared object to load: the built oracle, or a copy named by
    SGPM_ORACLE_LIB (the mutation tests load deliberately broken builds
    of this source that way, in a process of their own)."""
    return os.environ.get("SGPM_ORACLE_LIB") or _LIB


def lib():
    global _lib
    if _lib is None:
        path = lib_path()
        if path == _LIB and not os.path.exists(_LIB):
            build()
        L = C.CDLL(path)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint32)
        lp = C.POINTER(C.c_long)
        llp = C.POINTER(C.c_longlong)
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Params)]
        L.orc_destroy.argtypes = [P]
        L.orc_P.argtypes = [P]; L.orc_P.restype = C.c_int
        L.orc_Q.argtypes = [P]; L.orc_Q.restype = C.c_int
        L.orc_step_count.argtypes = [P]; L.orc_step_count.restype = C.c_long
        L.orc_set_threads.argtypes = [P, C.c_int]
        L.orc_init.argtypes = [P]
        L.orc_run.argtypes = [P, C.c_double, C.c_int, dp, up]
        L.orc_tables.argtypes = [P, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_get_state.argtypes = [P, dp, dp]
        L.orc_set_state.argtypes = [P, dp, dp, C.c_long]
        L.orc_get_histogram.argtypes = [P, up, up]
        L.orc_set_histogram.argtypes = [P, up, up]
        L.orc_get_counters.argtypes = [P, llp]
        L.orc_moments.argtypes = [P, dp]
        L.orc_step_particles.argtypes = [P, lp, C.c_long, C.c_uint32, C.c_double, dp, dp, llp]
        L.orc_rates_at.argtypes = [P, C.c_int, dp, dp, C.c_long, dp]
        L.orc_theta_ac_many.argtypes = [dp, dp, C.c_long, dp]
        L.orc_fd_inverse_many.argtypes = [P, C.c_int, up, up, C.c_long, dp]
        L.orc_philox_many.argtypes = [up, up, C.c_long, up]
        L.orc_gauss_legendre.argtypes = [C.c_int, dp, dp]
        L.orc_legendre_orthonormal.argtypes = [C.c_int, C.c_double]
        L.orc_legendre_orthonormal.restype = C.c_double
        L.orc_edge_integral.argtypes = [C.c_double, C.c_double]
        L.orc_edge_integral.restype = C.c_double
        L.orc_edge_angle.argtypes = [P, C.c_long, C.c_uint32, C.c_uint32, C.c_double, C.c_double]
        L.orc_edge_angle.restype = C.c_double
        L.orc_edge_kappa_coef.argtypes = [P]
        L.orc_edge_kappa_coef.restype = C.c_double
        L.orc_reconstruct_f.argtypes = [P, C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_reconstruct_f_at.argtypes = [P, dp, C.c_int, C.c_double, C.c_double, dp]
        L.orc_moments_at.argtypes = [P, C.c_int, dp, dp]
        L.orc_density_closed.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_density_closed.restype = C.c_double
        L.orc_init_particles.argtypes = [P, lp, C.c_long, dp, dp]
        L.orc_pauli_lookup.argtypes = [P, C.c_int, C.c_double, C.c_double, C.c_double]
        L.orc_pauli_lookup.restype = C.c_double
        L.orc_u52.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_u52.restype = C.c_double
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


DEFAULTS = dict(dim_z=0, degree=0, nodes_1d=1, n_particles=1000, gap_mode=0, gap_dim=-1,
                gap0=0.2, gap_rel=0.0, field_dim=-1, field0=1e6, field_rel=0.0,
                fermi_eV=0.4, temp_K=300.0, alpha=0.1, nk=240, lk_eV=5.0, pauli=1,
                final_state=0, rate_scale=(1.0,) * 6, seed=1, instance=0, c_max=32, splitting=0,
                init_temp_K=0.0)


def _params(cfg: dict) -> _Params:
    d = dict(DEFAULTS)
    d.update({k: v for k, v in cfg.items() if k in DEFAULTS})
    p = _Params()
    for k, v in d.items():
        if k == "rate_scale":
            p.rate_scale = (C.c_double * 6)(*[float(x) for x in v])
        else:
            setattr(p, k, v)
    return p


# ---------------------------------------------------------------- free helpers
def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    lib().orc_philox_many(_up(ctr), _up(key), ctr.shape[0], _up(out))
    return out


def uniform(whi: int, wlo: int) -> float:
    """(m + 1/2) 2^-52 with m the top 52 bits of (whi, wlo)."""
    return lib().orc_u52(whi, wlo)


def gauss_legendre(n: int):
    x = np.zeros(n); w = np.zeros(n)
    lib().orc_gauss_legendre(n, _dp(x), _dp(w))
    return x, w


def legendre_orthonormal(k: int, x: float) -> float:
    return lib().orc_legendre_orthonormal(k, x)


def density_closed(e0: float, mu: float, kT: float) -> float:
    """Equilibrium electron density (1/m^2) of a band with minimum e0, closed form."""
    return lib().orc_density_closed(e0, mu, kT, 6.62607015e-34 / (2 * np.pi))


def edge_integral(kap: float, c: float) -> float:
    return lib().orc_edge_integral(kap, c)


def theta_ac(u1: np.ndarray, u2: np.ndarray) -> np.ndarray:
    u1 = np.ascontiguousarray(u1, dtype=np.float64); u2 = np.ascontiguousarray(u2, dtype=np.float64)
    out = np.zeros_like(u1)
    lib().orc_theta_ac_many(_dp(u1), _dp(u2), u1.size, _dp(out))
    return out


# ------------------------------------------------------------------ simulation
class OracleSim:
    """One sG-PM instance on the CPU (FP64, sequential unless threads > 1)."""

    def __init__(self, cfg: dict, threads: int = 1):
        self.cfg = dict(cfg)
        self._p = _params(cfg)
        self._h = lib().orc_create(C.byref(self._p))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self.P = lib().orc_P(self._h)
        self.Q = lib().orc_Q(self._h)
        self.N = int(self._p.n_particles)
        self.nk = int(self._p.nk)
        lib().orc_set_threads(self._h, threads)
        self.record = []   # list of [Q][3] per recorded time

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # tables
    def tables(self) -> dict:
        P, Q = self.P, self.Q
        t = {k: np.zeros(n) for k, n in (("z", Q * 2), ("w", Q), ("psi", Q * P), ("ehat", P),
                                          ("eps0", Q), ("width", Q), ("field", Q), ("density", Q))}
        lib().orc_tables(self._h, *[_dp(t[k]) for k in ("z", "w", "psi", "ehat", "eps0", "width",
                                                          "field", "density")])
        t["z"] = t["z"].reshape(Q, 2); t["psi"] = t["psi"].reshape(Q, P)
        return t

    def init(self):
        lib().orc_init(self._h)
        self.record = [self.moments()]
        self.excess = [np.zeros(self.Q, dtype=np.uint32)]

    def run(self, dt: float, n_steps: int):
        out = np.zeros((n_steps, self.Q, 3))
        ex = np.zeros((n_steps, self.Q), dtype=np.uint32)
        lib().orc_run(self._h, dt, n_steps, _dp(out), _up(ex))
        self.record.extend(list(out))
        self.excess.extend(list(ex))
        return out

    @property
    def step_count(self) -> int:
        return lib().orc_step_count(self._h)

    def moments(self) -> np.ndarray:
        out = np.zeros((self.Q, 3))
        lib().orc_moments(self._h, _dp(out))
        return out

    def get_state(self):
        kx = np.zeros((self.P, self.N)); ky = np.zeros((self.P, self.N))
        lib().orc_get_state(self._h, _dp(kx), _dp(ky))
        return kx, ky

    def set_state(self, kx, ky, step: int = 0):
        kx = np.ascontiguousarray(kx, dtype=np.float64).reshape(self.P, self.N)
        ky = np.ascontiguousarray(ky, dtype=np.float64).reshape(self.P, self.N)
        lib().orc_set_state(self._h, _dp(kx), _dp(ky), step)
        self.record = [self.moments()]
        self.excess = [np.zeros(self.Q, dtype=np.uint32)]

    def histogram(self):
        H = np.zeros((self.Q, self.nk, self.nk), dtype=np.uint32)
        M = np.zeros(self.Q, dtype=np.uint32)
        lib().orc_get_histogram(self._h, _up(H), _up(M))
        return H, M

    def set_histogram(self, H, M):
        H = np.ascontiguousarray(H, dtype=np.uint32); M = np.ascontiguousarray(M, dtype=np.uint32)
        lib().orc_set_histogram(self._h, _up(H), _up(M))

    def counters(self) -> dict:
        out = (C.c_longlong * 6)()
        lib().orc_get_counters(self._h, out)
        names = ("collisions", "events", "pauli_rejected", "edge_exhausted", "cmax_hits",
                 "out_of_grid")
        return dict(zip(names, list(out)))

    def step_particles(self, idx, kx, ky, step: int, dt: float):
        """Step the given particles (coefficients [count][P] at t^n) with the
        histogram currently held.  Returns new (kx, ky, ncoll)."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        kx = np.array(kx, dtype=np.float64, order="C").reshape(len(idx), self.P)
        ky = np.array(ky, dtype=np.float64, order="C").reshape(len(idx), self.P)
        nc = np.zeros(len(idx), dtype=np.int64)
        lib().orc_step_particles(self._h, idx.ctypes.data_as(C.POINTER(C.c_long)), len(idx),
                                 step, dt, _dp(kx), _dp(ky),
                                 nc.ctypes.data_as(C.POINTER(C.c_longlong)))
        return kx, ky, nc

    def rates(self, q: int, kx, ky) -> np.ndarray:
        kx = np.ascontiguousarray(kx, dtype=np.float64).ravel()
        ky = np.ascontiguousarray(ky, dtype=np.float64).ravel()
        out = np.zeros((kx.size, 6))
        lib().orc_rates_at(self._h, q, _dp(kx), _dp(ky), kx.size, _dp(out))
        return out

    def fd_inverse(self, q: int, whi, wlo) -> np.ndarray:
        whi = np.ascontiguousarray(whi, dtype=np.uint32); wlo = np.ascontiguousarray(wlo, dtype=np.uint32)
        out = np.zeros(whi.size)
        lib().orc_fd_inverse_many(self._h, q, _up(whi), _up(wlo), whi.size, _dp(out))
        return out

    def edge_angle(self, i: int, step: int, coll: int, kx: float, ky: float) -> float:
        return lib().orc_edge_angle(self._h, i, step, coll, kx, ky)

    def init_particles(self, idx):
        """Initial coefficients of the listed particles, [count][P] each."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        kx = np.zeros((len(idx), self.P)); ky = np.zeros((len(idx), self.P))
        lib().orc_init_particles(self._h, idx.ctypes.data_as(C.POINTER(C.c_long)), len(idx),
                                 _dp(kx), _dp(ky))
        return kx, ky

    def pauli_lookup(self, q: int, kx: float, ky: float, dt: float) -> float:
        return lib().orc_pauli_lookup(self._h, q, kx, ky, dt)

    @property
    def edge_kappa_coef(self) -> float:
        return lib().orc_edge_kappa_coef(self._h)

    def reconstruct_f(self, nbins: int, emin: float, emax: float):
        nodes = np.zeros((self.Q, nbins)); modes = np.zeros((self.P, nbins))
        lib().orc_reconstruct_f(self._h, nbins, emin, emax, _dp(nodes), _dp(modes))
        return nodes, modes

    def reconstruct_f_at(self, z, nbins: int, emin: float, emax: float):
        zr = np.ravel(np.asarray(z, dtype=np.float64))
        z = np.zeros(2)
        z[:zr.size] = zr
        out = np.zeros(nbins)
        lib().orc_reconstruct_f_at(self._h, _dp(z), nbins, emin, emax, _dp(out))
        return out

    # ------------------------------------------------ quantities of interest
    def moments_at(self, z) -> dict:
        """V_x, V_y, mean energy, J_x of the particle expansion at points z."""
        dz = int(self.cfg.get("dim_z", 0))
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64).reshape(-1, max(dz, 1)))
        out = np.zeros((z.shape[0], 4))
        lib().orc_moments_at(self._h, z.shape[0], _dp(z), _dp(out))
        return {"V_x": out[:, 0], "V_y": out[:, 1], "energy": out[:, 2], "J_x": out[:, 3]}

    def qoi(self, rec=None) -> dict:
        """Expectation and variance over z (nodal quadrature) of V_x, J_x and
        the mean energy, for every recorded time (Sec. 4.2)."""
        t = self.tables()
        rec = np.asarray(self.record if rec is None else rec)   # [T][Q][3]
        w = t["w"]
        vx = rec[:, :, 0]
        en = rec[:, :, 2]
        jx = -Q_E * t["density"][None, :] * vx
        out = {}
        for name, x in (("vx", vx), ("jx", jx), ("energy", en)):
            m = x @ w
            out["E_" + name] = m
            out["Var_" + name] = ((x - m[:, None]) ** 2) @ w
        out["per_node_vx"] = vx
        out["per_node_energy"] = en
        out["per_node_jx"] = jx
        return out
