"""ctypes binding of libpolydg (include/pdg.h): argument marshalling only.

Every step of the residual, the time integration, the Hilbert keys and the partition runs in
the library's HIP kernels.  PyTorch supplies device memory and the HIP stream.  The binding
fails loudly when the built library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolydg.so")

PDG_OK, PDG_EINVAL, PDG_ENOMEM, PDG_EHIP, PDG_EMESH, PDG_ENOTSUP, PDG_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
EULER, NAVIER_STOKES = 0, 1

EXPORTED = (
    "pdg_create", "pdg_destroy", "pdg_layout", "pdg_node_coords", "pdg_project", "pdg_nodal",
    "pdg_residual", "pdg_rk_steps", "pdg_vjp", "pdg_vjp_static", "pdg_rk_stage", "pdg_rk_stage_adjoint",
    "pdg_nodal_adjoint", "pdg_node_weights", "pdg_sfc_keys", "pdg_partition",
    "pdg_set_schedule", "pdg_measure_costs", "pdg_type_weights", "pdg_batch_create", "pdg_batch_destroy",
    "pdg_batch_rk_steps", "pdg_batch_set_tiles", "pdg_batch_get_tiles", "pdg_batch_autotune",
    "pdg_batch_set_solo", "pdg_batch_get_solo",
    "pdg_timing_start", "pdg_timing_stop", "pdg_queue_times", "pdg_balance_weights", "pdg_rebalance",
    "pdg_get_schedule", "pdg_check_finite", "pdg_set_motion", "pdg_set_time", "pdg_get_time",
    "pdg_last_error",
)


class PdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libpolydg error {code}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [
        ("n_elems", ctypes.c_int32),
        ("n_vertices", ctypes.c_int32),
        ("elem_type", ctypes.c_void_p),
        ("elem_corner", ctypes.c_void_p),
        ("corner_xyz", ctypes.c_void_p),
        ("centroid", ctypes.c_void_p),
    ]


class _Params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32),
        ("equations", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("node_family", ctypes.c_int32),
        ("volume_form", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("Pr", ctypes.c_double),
        ("R", ctypes.c_double),
        ("p_ref", ctypes.c_double),
    ]


_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libpolydg.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "pdg_create": ([ctypes.POINTER(_Mesh), ctypes.POINTER(_Params), vp, ctypes.POINTER(vp)], ctypes.c_int),
        "pdg_destroy": ([vp], None),
        "pdg_layout": ([vp, ctypes.POINTER(i64), vp, vp, vp, vp], ctypes.c_int),
        "pdg_node_coords": ([vp, vp], ctypes.c_int),
        "pdg_project": ([vp, vp, vp], ctypes.c_int),
        "pdg_nodal": ([vp, vp, vp], ctypes.c_int),
        "pdg_residual": ([vp, vp, vp], ctypes.c_int),
        "pdg_rk_steps": ([vp, vp, vp, dbl, i32], ctypes.c_int),
        "pdg_vjp": ([vp, vp, vp, vp], ctypes.c_int),
        "pdg_vjp_static": ([vp, vp, vp, vp], ctypes.c_int),
        "pdg_rk_stage": ([vp, vp, vp, dbl, i32], ctypes.c_int),
        "pdg_timing_start": ([vp], ctypes.c_int),
        "pdg_timing_stop": ([vp, vp, vp], ctypes.c_int),
        "pdg_batch_create": ([vp, i32, vp, ctypes.POINTER(vp)], ctypes.c_int),
        "pdg_batch_destroy": ([vp], None),
        "pdg_batch_rk_steps": ([vp, vp, vp, vp, i32], ctypes.c_int),
        "pdg_batch_set_tiles": ([vp, vp], ctypes.c_int),
        "pdg_batch_get_tiles": ([vp, vp], ctypes.c_int),
        "pdg_batch_autotune": ([vp, vp, vp, vp, i32, vp], ctypes.c_int),
        "pdg_batch_set_solo": ([vp, i32], ctypes.c_int),
        "pdg_batch_get_solo": ([vp, ctypes.POINTER(i32)], ctypes.c_int),
        "pdg_rk_stage_adjoint": ([vp, vp, vp, vp, dbl, i32], ctypes.c_int),
        "pdg_nodal_adjoint": ([vp, vp, vp], ctypes.c_int),
        "pdg_node_weights": ([vp, vp], ctypes.c_int),
        "pdg_sfc_keys": ([vp, ctypes.POINTER(dbl), dbl, vp], ctypes.c_int),
        "pdg_partition": ([vp, vp, i32, vp], ctypes.c_int),
        "pdg_set_schedule": ([vp, vp, i32], ctypes.c_int),
        "pdg_measure_costs": ([vp, vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl)], ctypes.c_int),
        "pdg_type_weights": ([vp, ctypes.POINTER(dbl), vp, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
        "pdg_queue_times": ([vp, vp, i32, ctypes.POINTER(i64)], ctypes.c_int),
        "pdg_balance_weights": ([i32, vp, i32, vp, vp, vp, vp, ctypes.POINTER(dbl)], ctypes.c_int),
        "pdg_rebalance": ([vp, dbl, ctypes.POINTER(dbl)], ctypes.c_int),
        "pdg_get_schedule": ([vp, vp, ctypes.POINTER(i32)], ctypes.c_int),
        "pdg_check_finite": ([vp, vp, ctypes.POINTER(i64)], ctypes.c_int),
        "pdg_set_motion": ([vp, ctypes.POINTER(dbl), dbl], ctypes.c_int),
        "pdg_set_time": ([vp, dbl], ctypes.c_int),
        "pdg_get_time": ([vp, ctypes.POINTER(dbl)], ctypes.c_int),
        "pdg_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _LIB = lib
    return lib


def _check(rc):
    if rc != PDG_OK:
        msg = load_library().pdg_last_error().decode(errors="replace")
        raise PdgError(rc, msg)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def balance_weights(elem_type, queue_begin, queue_ms):
    """Element weights from measured per-queue times (host only, pdg_balance_weights).

    elem_type: int8 [n] in stored order; queue_begin: [Q+1]; queue_ms: [3, Q] (phase, queue).
    Returns (uint32 weights [n], fitted cost per element [3 phases, 4 types], imbalance)."""
    lib = load_library()
    et = np.ascontiguousarray(elem_type, dtype=np.int8)
    qb = np.ascontiguousarray(queue_begin, dtype=np.int32)
    ms = np.ascontiguousarray(queue_ms, dtype=np.float64)
    nq = qb.shape[0] - 1
    if ms.size != 3 * max(nq, 0):
        raise ValueError("queue_ms must hold 3 x n_queues values")
    w = np.empty(et.shape[0], dtype=np.uint32)
    tc = np.empty(12, dtype=np.float64)
    imb = ctypes.c_double()
    _check(lib.pdg_balance_weights(int(et.shape[0]), et.ctypes.data, int(nq), qb.ctypes.data, ms.ctypes.data,
                                   w.ctypes.data, tc.ctypes.data, ctypes.byref(imb)))
    return w, tc.reshape(3, 4), imb.value


class PolyDG:
    """A libpolydg context on the current CUDA (HIP) device and stream.

    Mesh arrays follow include/pdg.h (pdg_mesh); state tensors are float64 on the device in
    the library's layout (Hilbert element order, see `perm` and `offset`)."""

    def __init__(self, elem_type, elem_corner, corner_xyz, centroid, n_vertices, N,
                 equations="euler", gamma=1.4, mu=1.0 / 1600.0, Pr=0.71, R=1.0, p_ref=0.0,
                 stream=None, volume_form="weak", flux="lf"):
        import torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libpolydg needs a HIP device")
        self._arrays = dict(
            elem_type=np.ascontiguousarray(elem_type, dtype=np.int8),
            elem_corner=np.ascontiguousarray(elem_corner, dtype=np.int32),
            corner_xyz=np.ascontiguousarray(corner_xyz, dtype=np.float64),
            centroid=np.ascontiguousarray(centroid, dtype=np.float64),
        )
        a = self._arrays
        ne = a["elem_type"].shape[0]
        mesh = _Mesh(ne, int(n_vertices), a["elem_type"].ctypes.data, a["elem_corner"].ctypes.data,
                     a["corner_xyz"].ctypes.data, a["centroid"].ctypes.data)
        eq = {"euler": EULER, "ns": NAVIER_STOKES}[equations]
        vf = {"weak": 0, "split": 1}[volume_form]
        fl = {"lf": 0, "ec": 1}[flux]
        params = _Params(int(N), eq, fl, 0, vf, float(gamma), float(mu), float(Pr), float(R), float(p_ref))
        self.stream = torch.cuda.current_stream() if stream is None else stream
        handle = ctypes.c_void_p()
        _check(self.lib.pdg_create(ctypes.byref(mesh), ctypes.byref(params),
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)))
        self.handle = handle
        self.N, self.n, self.equations = int(N), int(N) + 1, equations
        self.volume_form, self.flux = volume_form, flux
        self.n_elems = ne
        nd = ctypes.c_int64()
        self.perm = np.empty(ne, dtype=np.int32)
        self.offset = np.empty(ne + 1, dtype=np.int64)
        self.elem_type = np.empty(ne, dtype=np.int8)
        self.elem_sides = np.empty((ne, 2), dtype=np.int32)
        _check(self.lib.pdg_layout(self.handle, ctypes.byref(nd), self.perm.ctypes.data,
                                   self.offset.ctypes.data, self.elem_type.ctypes.data,
                                   self.elem_sides.ctypes.data))
        self.n_doubles = int(nd.value)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def from_mesh(cls, mesh, N, **kw):
        return cls(mesh.elem_type, mesh.elem_corner, mesh.corner_xyz, mesh.centroid,
                   mesh.n_vertices, N, **kw)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.pdg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ tensors
    def empty_state(self):
        import torch
        return torch.empty(self.n_doubles, dtype=torch.float64, device=self.device)

    def zeros_state(self):
        import torch
        return torch.zeros(self.n_doubles, dtype=torch.float64, device=self.device)

    def _chk_state(self, t, name):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != self.n_doubles:
            raise ValueError(f"{name}: expected a contiguous float64 device tensor of {self.n_doubles} values")

    # ------------------------------------------------------------------ calls
    def residual(self, U, out=None):
        self._chk_state(U, "U")
        out = self.empty_state() if out is None else out
        self._chk_state(out, "out")
        _check(self.lib.pdg_residual(self.handle, _ptr(U), _ptr(out)))
        return out

    def rk_steps(self, U, K, dt, n_steps):
        self._chk_state(U, "U")
        self._chk_state(K, "K")
        _check(self.lib.pdg_rk_steps(self.handle, _ptr(U), _ptr(K), float(dt), int(n_steps)))
        return U, K

    def vjp(self, U, cot, out=None):
        self._chk_state(U, "U")
        self._chk_state(cot, "cot")
        out = self.empty_state() if out is None else out
        self._chk_state(out, "out")
        _check(self.lib.pdg_vjp(self.handle, _ptr(U), _ptr(cot), _ptr(out)))
        return out

    def vjp_static(self, U, cot, out):
        """pdg_vjp_static: the VJP with the library's static workspace; `out` is required (the
        call allocates nothing)."""
        self._chk_state(U, "U")
        self._chk_state(cot, "cot")
        self._chk_state(out, "out")
        _check(self.lib.pdg_vjp_static(self.handle, _ptr(U), _ptr(cot), _ptr(out)))
        return out

    def rk_stage(self, U, K, dt, stage):
        self._chk_state(U, "U")
        self._chk_state(K, "K")
        _check(self.lib.pdg_rk_stage(self.handle, _ptr(U), _ptr(K), float(dt), int(stage)))
        return U, K

    def rk_stage_adjoint(self, U_s, Ubar, Kbar, dt, stage):
        for t, name in ((U_s, "U_s"), (Ubar, "Ubar"), (Kbar, "Kbar")):
            self._chk_state(t, name)
        _check(self.lib.pdg_rk_stage_adjoint(self.handle, _ptr(U_s), _ptr(Ubar), _ptr(Kbar), float(dt),
                                             int(stage)))
        return Ubar, Kbar

    def nodal_adjoint(self, qbar):
        """qbar: [n_elems, 5, n^3] (stored element order) -> V^T qbar in the state layout."""
        import torch
        qbar = qbar.contiguous()
        if qbar.dtype != torch.float64 or tuple(qbar.shape) != (self.n_elems, 5, self.n ** 3):
            raise ValueError("qbar: expected float64 [n_elems, 5, n^3]")
        U = self.empty_state()
        _check(self.lib.pdg_nodal_adjoint(self.handle, _ptr(qbar), _ptr(U)))
        return U

    def check_finite(self, U):
        """Raise PdgError (code PDG_ENONFINITE) naming the first stored index of a NaN or infinite
        entry of U; return None when U is finite."""
        self._chk_state(U, "U")
        first = ctypes.c_int64()
        _check(self.lib.pdg_check_finite(self.handle, _ptr(U), ctypes.byref(first)))

    def node_weights(self):
        """w_k J_k at the volume nodes: [n_elems, n^3], stored element order."""
        import torch
        wJ = torch.empty((self.n_elems, self.n ** 3), dtype=torch.float64, device=self.device)
        _check(self.lib.pdg_node_weights(self.handle, _ptr(wJ)))
        return wJ

    def node_coords(self):
        import torch
        x = torch.empty((self.n_elems, self.n ** 3, 3), dtype=torch.float64, device=self.device)
        _check(self.lib.pdg_node_coords(self.handle, _ptr(x)))
        return x

    def project(self, q):
        """q: [n_elems, 5, n^3] nodal values (stored element order) -> state."""
        import torch
        if q.dtype != torch.float64 or not q.is_cuda or tuple(q.shape) != (self.n_elems, 5, self.n ** 3):
            raise ValueError(f"q must be a float64 CUDA tensor of shape ({self.n_elems}, 5, {self.n ** 3})")
        q = q.contiguous()
        U = self.empty_state()
        _check(self.lib.pdg_project(self.handle, _ptr(q), _ptr(U)))
        return U

    def nodal(self, U):
        import torch
        self._chk_state(U, "U")
        q = torch.empty((self.n_elems, 5, self.n ** 3), dtype=torch.float64, device=self.device)
        _check(self.lib.pdg_nodal(self.handle, _ptr(U), _ptr(q)))
        return q

    def sfc_keys(self, lo, scale):
        import torch
        keys = torch.empty(self.n_elems, dtype=torch.int64, device=self.device)
        lo3 = (ctypes.c_double * 3)(*[float(v) for v in lo])
        _check(self.lib.pdg_sfc_keys(self.handle, lo3, float(scale), _ptr(keys)))
        return keys

    def partition(self, weight, n_queues):
        import torch
        w = weight.to(device=self.device, dtype=torch.int32).contiguous()
        qb = torch.empty(n_queues + 1, dtype=torch.int32, device=self.device)
        _check(self.lib.pdg_partition(self.handle, _ptr(w), int(n_queues), _ptr(qb)))
        return qb

    def set_motion(self, corner_disp, omega):
        """Move every corner as x0 + d sin(omega t); corner_disp (host) [n_elems][8][3] in input
        element order."""
        d = np.ascontiguousarray(corner_disp, dtype=np.float64)
        if d.shape != (self.n_elems, 8, 3):
            raise ValueError(f"corner_disp must be ({self.n_elems}, 8, 3)")
        _check(self.lib.pdg_set_motion(self.handle, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       float(omega)))

    def set_time(self, t):
        _check(self.lib.pdg_set_time(self.handle, float(t)))

    @property
    def time(self):
        t = ctypes.c_double()
        _check(self.lib.pdg_get_time(self.handle, ctypes.byref(t)))
        return t.value

    def set_schedule(self, queue_begin=None):
        import torch
        if queue_begin is None:
            _check(self.lib.pdg_set_schedule(self.handle, None, 0))
            return
        qb = queue_begin.to(device=self.device, dtype=torch.int32).contiguous()
        _check(self.lib.pdg_set_schedule(self.handle, _ptr(qb), int(qb.numel() - 1)))

    def measure_costs(self, U, reps=3):
        """(seconds per element per residual for each type, average launch ms [phase][type])."""
        self._chk_state(U, "U")
        c = (ctypes.c_double * 4)()
        ph = (ctypes.c_double * 12)()
        _check(self.lib.pdg_measure_costs(self.handle, _ptr(U), int(reps), c, ph))
        return np.array(list(c)), np.array(list(ph)).reshape(3, 4)

    def type_weights(self, cost_per_elem):
        """(device int32 view of the uint32 element weights [n_elems], host per-type weights [4])."""
        import torch
        c = (ctypes.c_double * 4)(*[float(v) for v in cost_per_elem])
        wt = (ctypes.c_uint32 * 4)()
        w = torch.empty(self.n_elems, dtype=torch.int32, device=self.device)
        _check(self.lib.pdg_type_weights(self.handle, c, _ptr(w), wt))
        return w, np.array(list(wt), dtype=np.uint32)

    def queue_times(self, reset=False):
        """(ms [3 phases, Q queues] accumulated by the queue kernels, residual evaluations)."""
        nq = self.n_queues()
        ms = np.empty(3 * nq, dtype=np.float64)
        n = ctypes.c_int64()
        _check(self.lib.pdg_queue_times(self.handle, ms.ctypes.data, int(bool(reset)), ctypes.byref(n)))
        return ms.reshape(3, nq), n.value

    def n_queues(self):
        """Queues of the installed schedule (0: per-type launches)."""
        n = ctypes.c_int32()
        _check(self.lib.pdg_get_schedule(self.handle, None, ctypes.byref(n)))
        return n.value

    def rebalance(self, threshold):
        """Threshold-triggered rebalance of the installed schedule (pdg_rebalance)."""
        info = (ctypes.c_double * 4)()
        _check(self.lib.pdg_rebalance(self.handle, float(threshold), info))
        return {"imbalance": info[0], "predicted": info[1], "rebalanced": bool(info[2]),
                "evaluations": int(info[3])}

    def rk_steps_balanced(self, U, K, dt, n_steps, interval, threshold):
        """LSERK4 steps on the installed work-queue schedule with the dynamic balance loop: after
        every `interval` steps the queue timers of those steps decide on a rebalance.  Returns
        the rebalance records."""
        if interval <= 0:
            raise ValueError("interval must be positive")
        self.queue_times(reset=True)
        log, done = [], 0
        while done < n_steps:
            k = min(interval, n_steps - done)
            self.rk_steps(U, K, dt, k)
            done += k
            if done < n_steps:
                log.append(self.rebalance(threshold))
        return log

    def schedule(self):
        """Installed queue_begin as a host int32 array, or None (per-type launches)."""
        nq = self.n_queues()
        if nq == 0:
            return None
        qb = np.empty(nq + 1, dtype=np.int32)
        n = ctypes.c_int32()
        _check(self.lib.pdg_get_schedule(self.handle, qb.ctypes.data, ctypes.byref(n)))
        return qb

    def timing_start(self):
        _check(self.lib.pdg_timing_start(self.handle))

    def timing_stop(self):
        """(total ms, launches), each [3 phases][4 types], of the launches since timing_start."""
        ms = (ctypes.c_double * 12)()
        n = (ctypes.c_int32 * 12)()
        _check(self.lib.pdg_timing_stop(self.handle, ms, n))
        return np.array(list(ms)).reshape(3, 4), np.array(list(n)).reshape(3, 4)

    # ------------------------------------------------------------------ layout helpers
    def input_offsets(self):
        """Offsets of a state laid out in INPUT element order with the same per-element blocks."""
        sizes = np.diff(self.offset)
        in_sizes = np.empty_like(sizes)
        in_sizes[self.perm] = sizes
        return np.concatenate([[0], np.cumsum(in_sizes)]).astype(np.int64)

    def _gather_index(self):
        if not hasattr(self, "_gidx"):
            ioff = self.input_offsets()
            sizes = np.diff(self.offset)
            starts = ioff[self.perm]
            rep = np.repeat(starts - self.offset[:-1], sizes)
            self._gidx = (np.arange(self.n_doubles, dtype=np.int64) + rep)
        return self._gidx

    def from_input_order(self, x):
        """numpy state in input element order -> numpy state in library order."""
        return np.asarray(x)[self._gather_index()]

    def to_input_order(self, x):
        out = np.empty(self.n_doubles, dtype=np.float64)
        out[self._gather_index()] = np.asarray(x)
        return out


class PolyBatch:
    """Batched LSERK4 stepping of several PolyDG problems (pdg_batch_*): one graph launch per
    step for all of them.  The PolyDG objects must outlive the batch."""

    def __init__(self, problems, stream=None):
        import torch
        self.lib = load_library()
        self.problems = list(problems)
        if not self.problems:
            raise ValueError("empty batch")
        self.device = self.problems[0].device
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        handles = (ctypes.c_void_p * len(self.problems))(*[p.handle for p in self.problems])
        h = ctypes.c_void_p()
        _check(self.lib.pdg_batch_create(handles, len(self.problems), ctypes.c_void_p(stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pdg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _arrays(self, Us, Ks, dts):
        n = len(self.problems)
        if not (len(Us) == len(Ks) == len(dts) == n):
            raise ValueError("one U, K and dt per problem")
        for p, U, K in zip(self.problems, Us, Ks):
            p._chk_state(U, "U")
            p._chk_state(K, "K")
        Ua = (ctypes.c_void_p * n)(*[U.data_ptr() for U in Us])
        Ka = (ctypes.c_void_p * n)(*[K.data_ptr() for K in Ks])
        da = (ctypes.c_double * n)(*[float(d) for d in dts])
        return Ua, Ka, da

    def rk_steps(self, Us, Ks, dts, n_steps):
        Ua, Ka, da = self._arrays(Us, Ks, dts)
        _check(self.lib.pdg_batch_rk_steps(self.handle, Ua, Ka, da, int(n_steps)))

    def set_tiles(self, tiles):
        t = np.ascontiguousarray(np.asarray(tiles, dtype=np.int32).reshape(4, 7))
        _check(self.lib.pdg_batch_set_tiles(self.handle, t.ctypes.data_as(ctypes.c_void_p)))

    def tiles(self):
        t = np.zeros((4, 7), dtype=np.int32)
        _check(self.lib.pdg_batch_get_tiles(self.handle, t.ctypes.data_as(ctypes.c_void_p)))
        return t

    def set_solo(self, min_elems):
        """Problems with at least min_elems elements run alone (2**31 - 1: all merged)."""
        _check(self.lib.pdg_batch_set_solo(self.handle, int(min_elems)))

    def solo(self):
        v = ctypes.c_int32()
        _check(self.lib.pdg_batch_get_solo(self.handle, ctypes.byref(v)))
        return v.value

    def autotune(self, Us, Ks, dts, reps=3):
        Ua, Ka, da = self._arrays(Us, Ks, dts)
        t = np.zeros((4, 7), dtype=np.int32)
        _check(self.lib.pdg_batch_autotune(self.handle, Ua, Ka, da, int(reps), t.ctypes.data_as(ctypes.c_void_p)))
        return t
