"""MI355X (gfx950) implementation of the sG-PM hot path of arXiv:2404.19602.

A thin binding over the C-ABI library ``libsgpm.so`` (declared in
``include/sgpm.h``): argument marshalling only.  Every step of the particle
update runs in the library's HIP kernels; PyTorch provides the device
workspace and the stream.  There is no CPU fallback: if the library is not
built, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from ._lib import (AGG_NAMES, COUNTER_NAMES, KERNEL_NAMES, Desc, SgpmError, check, desc_from_cfg,
                   lib, LIB_PATH)

__all__ = ["Simulation", "philox_device", "SgpmError", "AGG_NAMES", "COUNTER_NAMES", "LIB_PATH"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the sG-PM library needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


class Simulation:
    """One or more sG-PM instances in one context on one GPU.

    ``cfgs``: a parameter dictionary or a list of them (keys as in
    ``sgpm_instance_desc``; see ``workloads``).  The device workspace is a
    torch uint8 tensor owned by this object; work is enqueued on ``stream``
    (default: the current torch stream of the device)."""

    def __init__(self, cfgs, device: int = 0, stream=None, max_steps: int | None = None):
        torch = _torch()
        if isinstance(cfgs, dict):
            cfgs = [cfgs]
        self.cfgs = [dict(c) for c in cfgs]
        self.n_inst = len(self.cfgs)
        self.device = torch.device("cuda", device)
        L = lib()
        arr = (Desc * self.n_inst)()
        for k, cfg in enumerate(self.cfgs):
            arr[k] = desc_from_cfg(cfg, max_steps)
        self._descs = arr
        nbytes = C.c_size_t(0)
        check(L.sgpm_workspace_bytes(arr, self.n_inst, C.byref(nbytes)), None, "workspace_bytes")
        self.workspace = torch.empty(max(int(nbytes.value), 256) + 256, dtype=torch.uint8,
                                     device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p(0)
        check(L.sgpm_create(arr, self.n_inst, C.c_void_p(aligned), C.c_size_t(nbytes.value),
                            C.c_void_p(self.stream.cuda_stream), C.byref(ctx)), None, "create")
        self._ctx = ctx
        self.sizes = []
        for k in range(self.n_inst):
            P = C.c_int32(); Q = C.c_int32()
            check(L.sgpm_sizes(ctx, k, C.byref(P), C.byref(Q)), ctx, "sizes")
            self.sizes.append((P.value, Q.value))
        self.P, self.Q = self.sizes[0]
        self.N = int(self.cfgs[0]["n_particles"])

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                self.stream.synchronize()
            except Exception:
                pass
            lib().sgpm_destroy(ctx)
            self._ctx = None

    # ---------------------------------------------------------------- calls
    def init_particles(self):
        check(lib().sgpm_init_particles(self._ctx), self._ctx, "init_particles")

    def step(self, n_steps: int = 1, dt: float | None = None):
        dt = self.cfgs[0].get("dt", 2e-15) if dt is None else dt
        check(lib().sgpm_step(self._ctx, C.c_double(dt), C.c_int64(n_steps)), self._ctx, "step")

    def last_step_ms(self) -> float:
        ms = C.c_double(0)
        check(lib().sgpm_last_step_ms(self._ctx, C.byref(ms)), self._ctx, "last_step_ms")
        return ms.value

    @property
    def step_count(self) -> int:
        s = C.c_int64(0)
        check(lib().sgpm_step_count(self._ctx, C.byref(s)), self._ctx, "step_count")
        return s.value

    def set_chunk(self, chunk: int, inst: int = 0):
        check(lib().sgpm_set_chunk(self._ctx, inst, chunk), self._ctx, "set_chunk")

    @staticmethod
    def _mode(on) -> int:
        return -1 if on is None else (1 if on else 0)

    def set_node_pairs(self, on):
        """The mirror-pair stream kernel (True), the generic one (False) or
        the automatic choice by particle count (None, the default) for the
        instances with one uncertain input; right after init/set_state."""
        check(lib().sgpm_set_node_pairs(self._ctx, self._mode(on)), self._ctx, "set_node_pairs")

    def set_collider_lanes(self, on):
        """A lane per candidate (True), a group of lanes per candidate (False)
        or the automatic choice by particle count (None, the default) in the
        collider of the instances with at most 12 nodes."""
        check(lib().sgpm_set_collider_lanes(self._ctx, self._mode(on)), self._ctx,
              "set_collider_lanes")

    def set_stream_lds(self, nbytes: int, inst: int = 0):
        """LDS bytes of a stream workgroup (sizes the histogram window); 0 = default."""
        check(lib().sgpm_set_stream_lds(self._ctx, inst, int(nbytes)), self._ctx, "set_stream_lds")

    def window(self, inst: int = 0) -> dict:
        w = C.c_int32(0); b = C.c_int32(0)
        check(lib().sgpm_window(self._ctx, inst, C.byref(w), C.byref(b)), self._ctx, "window")
        return {"cells": w.value, "lds_bytes": b.value}

    def node_pairs(self, inst: int = 0) -> bool:
        v = C.c_int32(0)
        check(lib().sgpm_node_pairs(self._ctx, inst, C.byref(v)), self._ctx, "node_pairs")
        return bool(v.value)

    def set_pair_block(self, alt: int):
        """0: the default workgroup size of the mirror-pair stream kernel; 1:
        the other one (the autotuner tries both)."""
        check(lib().sgpm_set_pair_block(self._ctx, int(alt)), self._ctx, "set_pair_block")

    def set_stream_nontemporal(self, mode):
        """True/False: non-temporal hints on the stream kernels' state access
        always / never; None: when some instance's state exceeds 1 GiB."""
        m = -1 if mode is None else (1 if mode else 0)
        check(lib().sgpm_set_stream_nontemporal(self._ctx, m), self._ctx, "set_stream_nontemporal")

    def stream_nontemporal(self) -> bool:
        v = C.c_int32(0)
        check(lib().sgpm_stream_nontemporal(self._ctx, C.byref(v)), self._ctx, "stream_nontemporal")
        return bool(v.value)

    def stream_threads(self, inst: int = 0) -> int:
        v = C.c_int32(0)
        check(lib().sgpm_stream_threads(self._ctx, inst, C.byref(v)), self._ctx, "stream_threads")
        return int(v.value)

    def collider_lanes(self, inst: int = 0) -> bool:
        v = C.c_int32(0)
        check(lib().sgpm_collider_lanes(self._ctx, inst, C.byref(v)), self._ctx, "collider_lanes")
        return bool(v.value)

    def set_graph(self, steps_per_graph: int):
        """0: launch every kernel; B >= 1: replay captured graphs of B steps."""
        check(lib().sgpm_set_graph(self._ctx, steps_per_graph), self._ctx, "set_graph")

    def set_profiling(self, on: bool):
        check(lib().sgpm_set_profiling(self._ctx, 1 if on else 0), self._ctx, "set_profiling")

    def autotune(self, trial_steps: int = 20, dt: float | None = None) -> float:
        """Pick the fastest launch shape (chunk scale and collider workgroups)
        from timed trials; the state is put back.  Returns ms per step."""
        dt = self.cfgs[0].get("dt", 2e-15) if dt is None else dt
        ms = C.c_double(0)
        check(lib().sgpm_autotune(self._ctx, C.c_double(dt), trial_steps, C.byref(ms)), self._ctx,
              "autotune")
        return ms.value

    def launch_shape(self, inst: int = 0) -> dict:
        ch = C.c_int32(); nw = C.c_int32(); g2 = C.c_int32()
        check(lib().sgpm_launch_shape(self._ctx, inst, C.byref(ch), C.byref(nw), C.byref(g2)),
              self._ctx, "launch_shape")
        return {"chunk": ch.value, "stream_workgroups": nw.value, "collider_workgroups": g2.value}

    def kernel_times(self) -> dict:
        """Mean device time (ms) and launch count of each step kernel over the
        last profiled step call."""
        ms = np.zeros(len(KERNEL_NAMES))
        n = np.zeros(len(KERNEL_NAMES), dtype=np.int64)
        check(lib().sgpm_kernel_times(self._ctx, ms.ctypes.data_as(C.c_void_p),
                                      n.ctypes.data_as(C.c_void_p)), self._ctx, "kernel_times")
        return {name: (float(ms[k]), int(n[k])) for k, name in enumerate(KERNEL_NAMES)}

    def moments(self, first: int = 0, count: int | None = None, inst: int = 0) -> dict:
        P, Q = self.sizes[inst]
        if count is None:
            count = self.record_length(inst) - first
        per = np.zeros((count, Q, 4))
        agg = np.zeros((count, len(AGG_NAMES)))
        check(lib().sgpm_moments(self._ctx, inst, first, count, per.ctypes.data_as(C.c_void_p),
                                 agg.ctypes.data_as(C.c_void_p)), self._ctx, "moments")
        out = {name: agg[:, k] for k, name in enumerate(AGG_NAMES)}
        out["per_node_vx"] = per[:, :, 0]
        out["per_node_vy"] = per[:, :, 1]
        out["per_node_energy"] = per[:, :, 2]
        out["per_node_jx"] = per[:, :, 3]
        return out

    def occupancy_excess(self, first: int = 0, count: int | None = None, inst: int = 0):
        """[count][Q] particles above the maximum occupation number per
        recorded time and node (Pauli violation)."""
        _, Q = self.sizes[inst]
        if count is None:
            count = self.record_length(inst) - first
        out = np.zeros((count, Q), dtype=np.uint32)
        check(lib().sgpm_occupancy_excess(self._ctx, inst, first, count,
                                          out.ctypes.data_as(C.c_void_p)), self._ctx,
              "occupancy_excess")
        return out

    def record_length(self, inst: int = 0) -> int:
        n = C.c_int64(0)
        check(lib().sgpm_record_length(self._ctx, inst, C.byref(n)), self._ctx, "record_length")
        return n.value

    def get_state(self, inst: int = 0):
        P, _ = self.sizes[inst]
        N = int(self.cfgs[inst]["n_particles"])
        buf = np.zeros(2 * P * N)
        check(lib().sgpm_get_state(self._ctx, inst, buf.ctypes.data_as(C.c_void_p)), self._ctx,
              "get_state")
        return buf[:P * N].reshape(P, N), buf[P * N:].reshape(P, N)

    def set_state(self, kx, ky, step: int = 0, inst: int = 0):
        P, _ = self.sizes[inst]
        N = int(self.cfgs[inst]["n_particles"])
        buf = np.concatenate([np.asarray(kx, dtype=np.float64).reshape(P * N),
                              np.asarray(ky, dtype=np.float64).reshape(P * N)])
        check(lib().sgpm_set_state(self._ctx, inst, buf.ctypes.data_as(C.c_void_p), step),
              self._ctx, "set_state")

    def histogram(self, inst: int = 0):
        _, Q = self.sizes[inst]
        nk = int(self.cfgs[inst].get("nk", 240))
        H = np.zeros((Q, nk, nk), dtype=np.uint32)
        M = np.zeros(Q, dtype=np.uint32)
        check(lib().sgpm_get_histogram(self._ctx, inst, H.ctypes.data_as(C.c_void_p),
                                       M.ctypes.data_as(C.c_void_p)), self._ctx, "get_histogram")
        return H, M

    def counters(self, inst: int = 0) -> dict:
        out = np.zeros(8, dtype=np.uint64)
        check(lib().sgpm_counters(self._ctx, inst, out.ctypes.data_as(C.c_void_p)), self._ctx,
              "counters")
        return {name: int(out[k]) for k, name in enumerate(COUNTER_NAMES)}

    def tables(self, inst: int = 0) -> dict:
        P, Q = self.sizes[inst]
        t = {k: np.zeros(n) for k, n in (("z", 2 * Q), ("w", Q), ("psi", Q * P), ("ehat", P),
                                          ("eps0", Q), ("width", Q), ("field", Q),
                                          ("density", Q))}
        check(lib().sgpm_tables(self._ctx, inst, *[t[k].ctypes.data_as(C.c_void_p) for k in
                                                   ("z", "w", "psi", "ehat", "eps0", "width",
                                                    "field", "density")]), self._ctx, "tables")
        t["z"] = t["z"].reshape(Q, 2)
        t["psi"] = t["psi"].reshape(Q, P)
        return t

    def reconstruct_f(self, nbins: int, emin: float, emax: float, inst: int = 0):
        P, Q = self.sizes[inst]
        nodes = np.zeros((Q, nbins)); modes = np.zeros((P, nbins))
        check(lib().sgpm_reconstruct_f(self._ctx, inst, nbins, C.c_double(emin), C.c_double(emax),
                                       nodes.ctypes.data_as(C.c_void_p),
                                       modes.ctypes.data_as(C.c_void_p)), self._ctx,
              "reconstruct_f")
        return nodes, modes

    def reconstruct_f_at(self, z, nbins: int, emin: float, emax: float, inst: int = 0):
        dz = int(self.cfgs[inst].get("dim_z", 0))
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64).reshape(-1, max(dz, 1))[:, :dz]
                                 if dz else np.zeros((np.size(z) if np.ndim(z) else 1, 0)))
        nz = z.shape[0]
        out = np.zeros((nz, nbins))
        check(lib().sgpm_reconstruct_f_at(self._ctx, inst, nz, z.ctypes.data_as(C.c_void_p), nbins,
                                          C.c_double(emin), C.c_double(emax),
                                          out.ctypes.data_as(C.c_void_p)), self._ctx,
              "reconstruct_f_at")
        return out

    def moments_at(self, z, inst: int = 0) -> dict:
        """V_x, V_y, mean energy and J_x of the particle expansion at points z
        ([n_z][dim_z]; a plain list of scalars for one uncertain input)."""
        dz = int(self.cfgs[inst].get("dim_z", 0))
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64).reshape(-1, max(dz, 1)))
        nz = z.shape[0]
        out = np.zeros((nz, 4))
        check(lib().sgpm_moments_at(self._ctx, inst, nz, z.ctypes.data_as(C.c_void_p),
                                    out.ctypes.data_as(C.c_void_p)), self._ctx, "moments_at")
        return {"V_x": out[:, 0], "V_y": out[:, 1], "energy": out[:, 2], "J_x": out[:, 3]}

    def inputs_at(self, z, inst: int = 0) -> dict:
        """The uncertain inputs at points z: band gap and band minimum (eV),
        ribbon width (m) and field (V/m)."""
        dz = int(self.cfgs[inst].get("dim_z", 0))
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64).reshape(-1, max(dz, 1)))
        nz = z.shape[0]
        out = np.zeros((nz, 4))
        check(lib().sgpm_inputs_at(self._ctx, inst, nz, z.ctypes.data_as(C.c_void_p),
                                   out.ctypes.data_as(C.c_void_p)), self._ctx, "inputs_at")
        return {"gap_eV": out[:, 0], "eps0_eV": out[:, 1], "width_m": out[:, 2],
                "field": out[:, 3]}

    def synchronize(self):
        self.stream.synchronize()


def philox_device(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Philox4x32-10 of the given counters and keys computed by the device."""
    torch = _torch()
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    n = ctr.shape[0]
    dc = torch.from_numpy(ctr.view(np.int32)).cuda()
    dk = torch.from_numpy(key.view(np.int32)).cuda()
    do = torch.empty_like(dc)
    s = torch.cuda.current_stream()
    check(lib().sgpm_philox_device(C.c_void_p(dc.data_ptr()), C.c_void_p(dk.data_ptr()),
                                   C.c_void_p(do.data_ptr()), C.c_int64(n),
                                   C.c_void_p(s.cuda_stream)), None, "philox_device")
    return do.cpu().numpy().view(np.uint32)
