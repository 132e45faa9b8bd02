"""MI355X-native Potential Difference Reduction (PDR) sweep for multicommodity-flow feasibility.

Thin ctypes binding over ``libpdr.so`` (the C ABI of ``include/pdr.h``). Every
step of a sweep runs in the library's HIP kernels; this module only marshals
arguments. It raises if the library is missing -- there is no CPU fallback.

To pass torch device tensors or torch streams, import torch before the first
use of this module: the library then binds to torch's HIP runtime (both carry
the same soname), so pointers and streams are shared. Loaded without torch it
uses the system ROCm runtime, and a torch imported afterwards would start a
second runtime that does not see the device.

Method: Liu, "A Localized Method for Multicommodity Flow Problem" (arXiv 2108.07549):
heights from excess (Section 3.1), the exact edge subproblem (PDR-ESO,
Section 4, Algorithms 1-2), the adaptive-gradient update (PDR-AGD,
Section 5.1, Algorithm 3), its momentum variant (PDR-GDM, Section 5.2,
Algorithm 4) and a capacity-enforcing loop for Section 6's formulation (CAP).
Batches: ``Batch``; the reverse-mode gradient: ``Context.adjoint`` and
``paper_2108_07549_amd.autograd``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdr.so")

ESO, AGD, GDM, CAP = 0, 1, 2, 3
FP64, FP32_BULK = 0, 1
VERDICT = {0: "undecided", 1: "feasible", 2: "infeasible"}
STATUS = {0: "PDR_OK", 1: "PDR_ERR_INVALID", 2: "PDR_ERR_OOM", 3: "PDR_ERR_DEVICE",
          4: "PDR_ERR_STATE", 5: "PDR_ERR_NUMERIC"}

EXPORTS = ["pdr_default_options", "pdr_init", "pdr_sweep", "pdr_solve", "pdr_residual", "pdr_flows",
           "pdr_flows_device", "pdr_stream", "pdr_heights", "pdr_learning_rates", "pdr_velocities", "pdr_z_log",
           "pdr_set_precision", "pdr_set_state", "pdr_set_state_noalloc", "pdr_profile_sweeps", "pdr_measure_copy",
           "pdr_tiling", "pdr_adjoint", "pdr_destroy", "pdr_last_error",
           "pdr_batch_init", "pdr_batch_sweep", "pdr_batch_member", "pdr_batch_stopped",
           "pdr_batch_tune", "pdr_batch_buckets", "pdr_batch_profile_sweeps",
           "pdr_batch_set_precision", "pdr_batch_last_error", "pdr_batch_destroy"]


class PdrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class AgdParams(C.Structure):
    _fields_ = [("beta_init", C.c_double), ("beta_min", C.c_double), ("beta_max", C.c_double),
                ("alpha_inc", C.c_double), ("alpha_dec", C.c_double), ("inc_period", C.c_int32),
                ("gamma", C.c_double)]


class Options(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("agd", AgdParams),
                ("gdm", AgdParams),
                ("z_feasible_tol", C.c_double), ("stream", C.c_void_p),
                ("lanes_per_arc", C.c_int32), ("vec_per_lane", C.c_int32),
                ("graph_sweeps", C.c_int32), ("height_chunk", C.c_int32),
                ("cluster_size", C.c_int32), ("height_blocks", C.c_int32),
                ("height_unroll", C.c_int32), ("z_log_capacity", C.c_int32),
                ("cache_policy", C.c_int32), ("batch_groups", C.c_int32),
                ("height_kernel", C.c_int32)]


class Residual(C.Structure):
    _fields_ = [("z", C.c_double), ("z_psi", C.c_double), ("z_h", C.c_double),
                ("kkt_sq", C.c_double), ("max_abs_excess", C.c_double),
                ("max_congestion", C.c_double), ("farkas_gap", C.c_double),
                ("farkas_tol", C.c_double), ("z_fp32_floor", C.c_double),
                ("sweeps_done", C.c_int64),
                ("evaluations", C.c_int64), ("verdict", C.c_int32), ("stopped", C.c_int32)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["verdict"] = VERDICT[int(self.verdict)]
        return d


class Instance(C.Structure):
    """pdr_instance: one instance of Section 1 for pdr_batch_init."""
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("u", C.c_void_p), ("K", C.c_int32),
                ("s", C.c_void_p), ("t", C.c_void_p), ("d", C.c_void_p)]


class BucketInfo(C.Structure):
    _fields_ = [("lanes_per_arc", C.c_int32), ("vec_per_lane", C.c_int32),
                ("instances", C.c_int32), ("max_K", C.c_int32), ("arcs", C.c_int64),
                ("ms", C.c_double)]


_lib = None


def lib():
    """Load libpdr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2108_07549_amd.build")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.pdr_default_options.argtypes = [C.POINTER(Options)]
        L.pdr_default_options.restype = None
        L.pdr_init.argtypes = [C.POINTER(P), i32, i32, P, P, P, i32, P, P, P, C.POINTER(Options)]
        L.pdr_sweep.argtypes = [P, i64, dbl, dbl]
        L.pdr_solve.argtypes = [P, dbl, i64, i64, dbl, C.POINTER(i64), C.POINTER(i64)]
        L.pdr_residual.argtypes = [P, C.POINTER(Residual)]
        L.pdr_flows.argtypes = [P, P]
        L.pdr_flows_device.argtypes = [P, P, i32]
        L.pdr_stream.argtypes = [P, C.POINTER(P)]
        L.pdr_heights.argtypes = [P, P]
        L.pdr_learning_rates.argtypes = [P, P]
        L.pdr_velocities.argtypes = [P, P]
        L.pdr_z_log.argtypes = [P, i64, i64, P]
        L.pdr_set_precision.argtypes = [P, i32]
        L.pdr_set_state.argtypes = [P, P, P, P, i64, dbl]
        L.pdr_set_state_noalloc.argtypes = [P, P, P, P, i64, dbl]
        L.pdr_profile_sweeps.argtypes = [P, i64, P]
        L.pdr_measure_copy.argtypes = [i64, i32, P]
        L.pdr_adjoint.argtypes = [P, i64, i32, P, P, P]
        L.pdr_tiling.argtypes = [P, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.pdr_destroy.argtypes = [P]
        L.pdr_destroy.restype = None
        L.pdr_last_error.argtypes = [P]
        L.pdr_last_error.restype = C.c_char_p
        L.pdr_batch_init.argtypes = [C.POINTER(P), i32, C.POINTER(Instance), C.POINTER(Options)]
        L.pdr_batch_sweep.argtypes = [P, i64, dbl, dbl]
        L.pdr_batch_member.argtypes = [P, i32, C.POINTER(P)]
        L.pdr_batch_stopped.argtypes = [P, C.POINTER(i32)]
        L.pdr_batch_tune.argtypes = [P, i32, C.POINTER(i64)]
        L.pdr_batch_buckets.argtypes = [P, i32, C.POINTER(BucketInfo), C.POINTER(i32)]
        L.pdr_batch_profile_sweeps.argtypes = [P, i64, P]
        L.pdr_batch_set_precision.argtypes = [P, i32]
        L.pdr_batch_last_error.argtypes = [P]
        L.pdr_batch_last_error.restype = C.c_char_p
        L.pdr_batch_destroy.argtypes = [P]
        L.pdr_batch_destroy.restype = None
        for name in EXPORTS:
            if name not in ("pdr_default_options", "pdr_destroy", "pdr_last_error",
                            "pdr_batch_last_error", "pdr_batch_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def measure_copy(nbytes: int = 4 << 30, iters: int = 10) -> float:
    """HBM bandwidth (GB/s, read + write) of a plain 16-byte copy kernel."""
    out = np.zeros(1, np.float64)
    st = lib().pdr_measure_copy(int(nbytes), int(iters), _ptr(out))
    if st != 0:
        raise PdrError(st, lib().pdr_last_error(None).decode())
    return float(out[0])


def device_synchronize():
    """hipDeviceSynchronize on the HIP runtime the library is bound to."""
    lib()
    hip = C.CDLL("libamdhip64.so.7")  # already loaded with the library: the same runtime
    st = hip.hipDeviceSynchronize()
    if st != 0:
        raise RuntimeError(f"hipDeviceSynchronize failed with error {st}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream: the HIP stream on ROCm


def default_options(method=ESO, precision=FP64, stream=None, lanes_per_arc=0, vec_per_lane=0,
                    z_feasible_tol=1e-8, agd=None, graph_sweeps=0, height_chunk=0,
                    cluster_size=0, height_blocks=0, height_unroll=0,
                    cache_policy=0, height_kernel=0) -> Options:
    opt = Options()
    lib().pdr_default_options(C.byref(opt))
    opt.method = int(method)
    opt.precision = int(precision)
    opt.stream = _stream_handle(stream)
    opt.lanes_per_arc = int(lanes_per_arc)
    opt.vec_per_lane = int(vec_per_lane)
    opt.z_feasible_tol = float(z_feasible_tol)
    opt.graph_sweeps = int(graph_sweeps)
    opt.height_chunk = int(height_chunk)
    opt.cluster_size = int(cluster_size)
    opt.height_blocks = int(height_blocks)
    opt.height_unroll = int(height_unroll)
    opt.cache_policy = int(cache_policy)
    opt.height_kernel = int(height_kernel)
    if agd:  # overrides for the AGD or GDM parameters of the chosen method
        target = opt.gdm if int(method) == GDM else opt.agd
        for k, v in agd.items():
            setattr(target, k, v)
    return opt


class Context:
    """One PDR instance resident on the GPU (wraps pdr_init ... pdr_destroy)."""

    def __init__(self, n, row_ptr, col, u, s, t, d, method=ESO, precision=FP64, stream=None,
                 lanes_per_arc=0, vec_per_lane=0, z_feasible_tol=1e-8, agd=None, graph_sweeps=0,
                 height_chunk=0, cluster_size=0, height_blocks=0, height_unroll=0,
                 cache_policy=0, height_kernel=0):
        L = lib()
        self._h = C.c_void_p()
        self._keep = [np.ascontiguousarray(row_ptr, np.int64), np.ascontiguousarray(col, np.int32),
                      np.ascontiguousarray(u, np.float64), np.ascontiguousarray(s, np.int32),
                      np.ascontiguousarray(t, np.int32), np.ascontiguousarray(d, np.float64)]
        rp, cl, uu, ss, tt, dd = self._keep
        self.n, self.m, self.K = int(n), int(cl.shape[0]), int(ss.shape[0])
        opt = default_options(method, precision, stream, lanes_per_arc, vec_per_lane,
                              z_feasible_tol, agd, graph_sweeps, height_chunk, cluster_size,
                              height_blocks, height_unroll, cache_policy, height_kernel)
        st = L.pdr_init(C.byref(self._h), int(n), self.m, _ptr(rp), _ptr(cl), _ptr(uu), self.K,
                        _ptr(ss), _ptr(tt), _ptr(dd), C.byref(opt))
        if st != 0:
            raise PdrError(st, L.pdr_last_error(None).decode())
        self._keep = None

    @classmethod
    def from_instance(cls, inst, **kw) -> "Context":
        return cls(inst.n, inst.row_ptr, inst.col, inst.u, inst.s, inst.t, inst.d, **kw)

    # -- helpers
    def _check(self, st):
        if st != 0:
            raise PdrError(st, lib().pdr_last_error(self._h).decode())

    @property
    def handle(self):
        return self._h

    # -- ABI mirror
    def sweep(self, max_sweeps: int, eps_obj: float = 0.0, z_target: float = 0.0):
        self._check(lib().pdr_sweep(self._h, int(max_sweeps), float(eps_obj), float(z_target)))

    def solve(self, z_target: float, max_sweeps: int, window: int = 256,
              floor_factor: float = 0.0):
        """Run to z <= z_target; FP32-bulk contexts switch to the FP64 polish near
        their rounding floor. Returns (passes in FP32, passes in FP64)."""
        a, b = C.c_int64(), C.c_int64()
        self._check(lib().pdr_solve(self._h, float(z_target), int(max_sweeps), int(window),
                                    float(floor_factor), C.byref(a), C.byref(b)))
        return a.value, b.value

    def residual(self) -> dict:
        r = Residual()
        st = lib().pdr_residual(self._h, C.byref(r))
        if st not in (0, 5):
            self._check(st)
        out = r.as_dict()
        out["status"] = STATUS[st]
        return out

    def flows(self) -> np.ndarray:
        out = np.empty((self.m, self.K), np.float64)
        self._check(lib().pdr_flows(self._h, _ptr(out)))
        return out

    def stream_handle(self) -> int:
        """The HIP stream (as an integer handle) the context's work runs on."""
        out = C.c_void_p()
        self._check(lib().pdr_stream(self._h, C.byref(out)))
        return int(out.value or 0)

    def flows_device(self, out_tensor, fp64: bool = True):
        """Write flows into a caller-owned device tensor of m*K elements
        (float64 when fp64, else float32), contiguous, on the context's GPU.
        The write is ordered after torch's current stream's earlier work on
        the tensor, and later work on that stream sees the flows: the context
        stream waits for torch's stream before the write, and torch's stream
        waits for the context stream after it (events, no host sync)."""
        import torch
        want = torch.float64 if fp64 else torch.float32
        if not out_tensor.is_cuda or out_tensor.dtype != want:
            raise ValueError(f"flows_device needs a {want} GPU tensor")
        if not out_tensor.is_contiguous() or out_tensor.numel() < self.m * self.K:
            raise ValueError(f"flows_device needs a contiguous tensor of at least "
                             f"m*K = {self.m * self.K} elements")
        cur = torch.cuda.current_stream(out_tensor.device)
        mine = torch.cuda.ExternalStream(self.stream_handle(), device=out_tensor.device)
        same = mine.cuda_stream == cur.cuda_stream
        if not same:
            mine.wait_stream(cur)
        self._check(lib().pdr_flows_device(self._h, C.c_void_p(out_tensor.data_ptr()),
                                           1 if fp64 else 0))
        if not same:
            cur.wait_stream(mine)
        return out_tensor

    def heights(self) -> np.ndarray:
        out = np.empty((self.n, self.K), np.float64)
        self._check(lib().pdr_heights(self._h, _ptr(out)))
        return out

    def learning_rates(self) -> np.ndarray:
        out = np.empty(self.m, np.float64)
        self._check(lib().pdr_learning_rates(self._h, _ptr(out)))
        return out

    def velocities(self) -> np.ndarray:
        out = np.empty((self.m, self.K), np.float64)
        self._check(lib().pdr_velocities(self._h, _ptr(out)))
        return out

    def z_log(self, first: int, count: int) -> np.ndarray:
        out = np.empty(max(int(count), 1), np.float64)
        self._check(lib().pdr_z_log(self._h, int(first), int(count), _ptr(out)))
        return out[:count]

    def set_precision(self, precision: int):
        self._check(lib().pdr_set_precision(self._h, int(precision)))

    def set_state(self, f, beta=None, t: int = 0, z_prev: float = float("inf"), v=None):
        fa = np.ascontiguousarray(f, np.float64)
        ba = None if beta is None else np.ascontiguousarray(beta, np.float64)
        va = None if v is None else np.ascontiguousarray(v, np.float64)
        self._check(lib().pdr_set_state(self._h, _ptr(fa), None if ba is None else _ptr(ba),
                                        None if va is None else _ptr(va), int(t), float(z_prev)))

    def set_state_noalloc(self, f, beta=None, t: int = 0, z_prev: float = float("inf"),
                          v=None):
        """set_state through pdr_set_state_noalloc (no device allocation)."""
        fa = np.ascontiguousarray(f, np.float64)
        ba = None if beta is None else np.ascontiguousarray(beta, np.float64)
        va = None if v is None else np.ascontiguousarray(v, np.float64)
        self._check(lib().pdr_set_state_noalloc(self._h, _ptr(fa),
                                                None if ba is None else _ptr(ba),
                                                None if va is None else _ptr(va), int(t),
                                                float(z_prev)))

    def profile_sweeps(self, sweeps: int) -> np.ndarray:
        """Run sweeps without a stop test; returns summed device ms of the
        (height + objective, arc) kernels measured with HIP events."""
        out = np.zeros(2, np.float64)
        self._check(lib().pdr_profile_sweeps(self._h, int(sweeps), _ptr(out)))
        return out

    def adjoint(self, T: int, checkpoint: int = 0):
        """T PDR-ESO passes (FP64) and the gradient of z(f^T) by reverse mode:
        returns (z, dz/du, dz/dd)."""
        z = np.zeros(1)
        gu = np.zeros(max(self.m, 1))
        gd = np.zeros(self.K)
        self._check(lib().pdr_adjoint(self._h, int(T), int(checkpoint), _ptr(z), _ptr(gu),
                                      _ptr(gd)))
        return float(z[0]), gu[:self.m], gd

    def tiling(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(lib().pdr_tiling(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def destroy(self):
        if self._h:
            lib().pdr_destroy(self._h)
            self._h = C.c_void_p()

    close = destroy

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """Many instances swept together (wraps pdr_batch_init ... pdr_batch_destroy).

    ``member(i)`` returns instance i's context (owned by the batch) for
    per-instance reads: flows, residual and verdict, z log."""

    def __init__(self, instances, method=ESO, precision=FP64, stream=None, agd=None,
                 graph_sweeps=0, z_log_capacity=0, lanes_per_arc=0, vec_per_lane=0,
                 height_blocks=0, groups=0, height_chunk=0):
        L = lib()
        self._h = C.c_void_p()
        keep, arr = [], (Instance * len(instances))()
        for q, inst in enumerate(instances):
            a = [np.ascontiguousarray(inst.row_ptr, np.int64),
                 np.ascontiguousarray(inst.col, np.int32), np.ascontiguousarray(inst.u, np.float64),
                 np.ascontiguousarray(inst.s, np.int32), np.ascontiguousarray(inst.t, np.int32),
                 np.ascontiguousarray(inst.d, np.float64)]
            keep.append(a)
            arr[q] = Instance(int(inst.n), int(a[1].shape[0]), _ptr(a[0]), _ptr(a[1]), _ptr(a[2]),
                              int(a[3].shape[0]), _ptr(a[3]), _ptr(a[4]), _ptr(a[5]))
        opt = default_options(method, precision, stream, lanes_per_arc, vec_per_lane, 1e-8, agd,
                              graph_sweeps)
        opt.z_log_capacity = int(z_log_capacity)
        opt.height_blocks = int(height_blocks)
        opt.batch_groups = int(groups)
        opt.height_chunk = int(height_chunk)
        st = L.pdr_batch_init(C.byref(self._h), len(instances), arr, C.byref(opt))
        if st != 0:
            raise PdrError(st, L.pdr_batch_last_error(None).decode())
        self.B = len(instances)
        self.sizes = [(int(i.n), int(i.m), int(i.K)) for i in instances]
        self._members = {}

    def _check(self, st):
        if st != 0:
            raise PdrError(st, lib().pdr_batch_last_error(self._h).decode())

    def sweep(self, max_sweeps: int, eps_obj: float = 0.0, z_target: float = 0.0):
        self._check(lib().pdr_batch_sweep(self._h, int(max_sweeps), float(eps_obj),
                                          float(z_target)))

    def member(self, index: int) -> "Context":
        if index not in self._members:
            h = C.c_void_p()
            self._check(lib().pdr_batch_member(self._h, int(index), C.byref(h)))
            ctx = Context.__new__(Context)
            ctx._h = h
            ctx._keep = None
            ctx.n, ctx.m, ctx.K = self.sizes[index]
            self._members[index] = ctx
        return self._members[index]

    def stopped(self) -> int:
        n = C.c_int32()
        self._check(lib().pdr_batch_stopped(self._h, C.byref(n)))
        return n.value

    def tune(self, reps: int = 5):
        """Autotune the arc tilings per bucket and the height launch; returns
        the buckets (with their tuned arc-kernel ms)."""
        hb = C.c_int64()
        self._check(lib().pdr_batch_tune(self._h, int(reps), C.byref(hb)))
        self.height_blocks = hb.value
        return self.buckets()

    def buckets(self):
        n = C.c_int32()
        self._check(lib().pdr_batch_buckets(self._h, 0, None, C.byref(n)))
        arr = (BucketInfo * max(n.value, 1))()
        self._check(lib().pdr_batch_buckets(self._h, n.value, arr, C.byref(n)))
        return [{name: getattr(arr[q], name) for name, _ in BucketInfo._fields_}
                for q in range(n.value)]

    def set_state_noalloc(self, f, beta=None, t: int = 0, z_prev: float = float("inf"),
                          v=None):
        """set_state through pdr_set_state_noalloc (no device allocation)."""
        fa = np.ascontiguousarray(f, np.float64)
        ba = None if beta is None else np.ascontiguousarray(beta, np.float64)
        va = None if v is None else np.ascontiguousarray(v, np.float64)
        self._check(lib().pdr_set_state_noalloc(self._h, _ptr(fa),
                                                None if ba is None else _ptr(ba),
                                                None if va is None else _ptr(va), int(t),
                                                float(z_prev)))

    def profile_sweeps(self, sweeps: int) -> np.ndarray:
        out = np.zeros(2, np.float64)
        self._check(lib().pdr_batch_profile_sweeps(self._h, int(sweeps), _ptr(out)))
        return out

    def set_precision(self, precision: int):
        self._check(lib().pdr_batch_set_precision(self._h, int(precision)))

    def destroy(self):
        if self._h:
            for ctx in self._members.values():
                ctx._h = C.c_void_p()
            self._members = {}
            lib().pdr_batch_destroy(self._h)
            self._h = C.c_void_p()

    close = destroy

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
