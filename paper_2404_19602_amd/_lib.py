"""ctypes declarations of the C-ABI in include/sgpm.h."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsgpm.so")

COUNTER_NAMES = ("collisions", "events", "pauli_rejected", "edge_exhausted", "cmax_hits",
                 "out_of_grid", "candidates", "reserved")
KERNEL_NAMES = ("stream", "finalize", "collide")
AGG_NAMES = ("E_vx", "Var_vx", "E_jx", "Var_jx", "E_energy", "Var_energy", "SE_E_vx",
             "SE_Var_vx", "SE_E_jx", "SE_Var_jx", "SE_E_energy", "SE_Var_energy")


class SgpmError(RuntimeError):
    pass


class Desc(C.Structure):
    """sgpm_instance_desc"""
    _fields_ = [
        ("dim_z", C.c_int32), ("degree", C.c_int32), ("nodes_1d", C.c_int32),
        ("precision", C.c_int32), ("n_particles", C.c_int64),
        ("gap_mode", C.c_int32), ("gap_dim", C.c_int32),
        ("gap0", C.c_double), ("gap_rel", C.c_double),
        ("field_dim", C.c_int32), ("field0", C.c_double), ("field_rel", C.c_double),
        ("fermi_eV", C.c_double), ("temp_K", C.c_double), ("alpha", C.c_double),
        ("nk", C.c_int32), ("lk_eV", C.c_double),
        ("pauli", C.c_int32), ("final_state", C.c_int32),
        ("rate_scale", C.c_double * 6),
        ("seed", C.c_uint64), ("instance_id", C.c_uint32), ("c_max", C.c_int32),
        ("max_steps", C.c_int32), ("splitting", C.c_int32),
        ("init_temp_K", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "sgpm_default_desc": (None, [C.POINTER(Desc)]),
            "sgpm_workspace_bytes": (i32, [C.POINTER(Desc), i32, C.POINTER(C.c_size_t)]),
            "sgpm_create": (i32, [C.POINTER(Desc), i32, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "sgpm_init_particles": (i32, [vp]),
            "sgpm_step": (i32, [vp, dbl, i64]),
            "sgpm_step_count": (i32, [vp, C.POINTER(i64)]),
            "sgpm_record_length": (i32, [vp, i32, C.POINTER(i64)]),
            "sgpm_moments": (i32, [vp, i32, i64, i64, vp, vp]),
            "sgpm_reconstruct_f": (i32, [vp, i32, i32, dbl, dbl, vp, vp]),
            "sgpm_reconstruct_f_at": (i32, [vp, i32, i32, vp, i32, dbl, dbl, vp]),
            "sgpm_moments_at": (i32, [vp, i32, i32, vp, vp]),
            "sgpm_inputs_at": (i32, [vp, i32, i32, vp, vp]),
            "sgpm_occupancy_excess": (i32, [vp, i32, i64, i64, vp]),
            "sgpm_set_state": (i32, [vp, i32, vp, i64]),
            "sgpm_get_state": (i32, [vp, i32, vp]),
            "sgpm_get_histogram": (i32, [vp, i32, vp, vp]),
            "sgpm_counters": (i32, [vp, i32, vp]),
            "sgpm_sizes": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32)]),
            "sgpm_tables": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
            "sgpm_set_chunk": (i32, [vp, i32, i32]),
            "sgpm_last_step_ms": (i32, [vp, C.POINTER(dbl)]),
            "sgpm_set_graph": (i32, [vp, i32]),
            "sgpm_set_node_pairs": (i32, [vp, i32]),
            "sgpm_set_collider_lanes": (i32, [vp, i32]),
            "sgpm_set_stream_lds": (i32, [vp, i32, i32]),
            "sgpm_window": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32)]),
            "sgpm_node_pairs": (i32, [vp, i32, C.POINTER(i32)]),
            "sgpm_collider_lanes": (i32, [vp, i32, C.POINTER(i32)]),
            "sgpm_set_pair_block": (i32, [vp, i32]),
            "sgpm_set_stream_nontemporal": (i32, [vp, i32]),
            "sgpm_stream_nontemporal": (i32, [vp, C.POINTER(i32)]),
            "sgpm_stream_threads": (i32, [vp, i32, C.POINTER(i32)]),
            "sgpm_set_profiling": (i32, [vp, i32]),
            "sgpm_kernel_times": (i32, [vp, vp, vp]),
            "sgpm_autotune": (i32, [vp, dbl, i32, C.POINTER(dbl)]),
            "sgpm_launch_shape": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
            "sgpm_destroy": (None, [vp]),
            "sgpm_last_error": (C.c_char_p, [vp]),
            "sgpm_status_string": (C.c_char_p, [i32]),
            "sgpm_philox_device": (i32, [vp, vp, vp, i64, vp]),
            "sgpm_energy_density_noalloc": (i32, [vp, vp, i32, i64, i32, i32, vp, vp, i32, dbl,
                                                  dbl, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, ctx, what: str):
    if status != 0:
        L = lib()
        msg = L.sgpm_status_string(status).decode()
        if ctx is not None:
            detail = L.sgpm_last_error(ctx)
            if detail:
                msg += ": " + detail.decode()
        raise SgpmError(f"sgpm {what} failed ({status}): {msg}")


_DEFAULTS = dict(dim_z=0, degree=0, nodes_1d=1, n_particles=10000, gap_mode=0, gap_dim=-1,
                 gap0=0.2, gap_rel=0.0, field_dim=-1, field0=1e6, field_rel=0.0, fermi_eV=0.4,
                 temp_K=300.0, alpha=0.1, nk=240, lk_eV=5.0, pauli=1, final_state=0,
                 rate_scale=(1.0,) * 6, seed=1, instance=0, c_max=32, splitting=0,
                 init_temp_K=0.0)


def desc_from_cfg(cfg: dict, max_steps: int | None = None) -> Desc:
    d = dict(_DEFAULTS)
    d.update({k: v for k, v in cfg.items() if k in _DEFAULTS})
    out = Desc()
    for k, v in d.items():
        if k == "rate_scale":
            out.rate_scale = (C.c_double * 6)(*[float(x) for x in v])
        elif k == "instance":
            out.instance_id = int(v)
        else:
            setattr(out, k, v)
    prec = cfg.get("precision", "fp64")
    out.precision = 1 if prec in ("fp32", 1) else 0
    steps = max_steps if max_steps is not None else int(cfg.get("max_steps", cfg.get("steps", 1000)))
    out.max_steps = int(steps)
    return out
