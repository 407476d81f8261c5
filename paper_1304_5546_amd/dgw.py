"""Thin ctypes binding over libdgw.so (argument marshalling only).

Every step of the solver runs in the HIP library; this module converts NumPy
arrays to the C ABI of ``include/dgw.h`` and raises ``DgwError`` on a negative
return code.  PyTorch is used only for streams and device buffers
(``set_fields_dev`` / ``get_fields_dev`` / ``launch_steps`` take tensors and a
``torch.cuda.Stream``).  Loading fails loudly when the in-tree library has not
been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DGW_LIB selects another build of the same library (the host-sanitizer
# build of the CPU tests); default: the in-tree libdgw.so
LIB_PATH = os.environ.get("DGW_LIB") or os.path.join(_HERE, "libdgw.so")

DGW_FP32, DGW_SPLIT_BF16, DGW_SPLIT_FP16, DGW_FP64 = 0, 1, 2, 3
PRECISIONS = {"fp32": DGW_FP32, "split_bf16": DGW_SPLIT_BF16, "split_fp16": DGW_SPLIT_FP16, "fp64": DGW_FP64}

ERRORS = {0: "DGW_OK", -1: "DGW_EINVAL", -2: "DGW_EMESH", -3: "DGW_EORDER", -4: "DGW_ENOMEM",
          -5: "DGW_ETOOBIG", -6: "DGW_EDEVICE", -7: "DGW_ENONFINITE", -8: "DGW_ECANCELLED",
          -9: "DGW_ENOTFOUND", -10: "DGW_ENODEVICE"}


class DgwError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({msg})")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_verts", C.c_int64), ("vx", C.c_void_p), ("vy", C.c_void_p),
                ("vz", C.c_void_p), ("n_elems", C.c_int64), ("elem_verts", C.c_void_p),
                ("eps", C.c_void_p), ("mu", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("alpha", C.c_double), ("cfl", C.c_double), ("prec", C.c_int32), ("renumber", C.c_int32),
                ("device", C.c_int32), ("kernel", C.c_int32), ("hip_stream", C.c_void_p),
                ("lane_elems", C.c_int32), ("wave_private", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("steps", C.c_int64), ("dt", C.c_double), ("t", C.c_double), ("setup_s", C.c_double),
                ("solve_ms", C.c_double), ("dof_updates_per_s", C.c_double), ("kernel", C.c_int32),
                ("groups_per_cu", C.c_int32), ("lane_elems", C.c_int32), ("wave_private", C.c_int32)]


TUNE_MAX = 24


class TuneInfo(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("groups_per_cu", C.c_int32), ("lane_elems", C.c_int32),
                ("wave_private", C.c_int32), ("best_us", C.c_double),
                ("n_tried", C.c_int32), ("tried_kernel", C.c_int32 * TUNE_MAX),
                ("tried_groups_per_cu", C.c_int32 * TUNE_MAX), ("tried_lane_elems", C.c_int32 * TUNE_MAX),
                ("tried_wave_private", C.c_int32 * TUNE_MAX), ("tried_us", C.c_double * TUNE_MAX)]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("device", C.c_int32),
                ("setup_threads", C.c_int32), ("max_chunk_steps", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("mesh", Mesh), ("order", C.c_int32), ("mode", C.c_int32 * 3), ("q0", C.c_void_p),
                ("t_final", C.c_double), ("alpha", C.c_double), ("prec", C.c_int32), ("keep_fields", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("order", C.c_int32), ("K", C.c_int64), ("steps", C.c_int64),
                ("dt", C.c_double), ("energy", C.c_double), ("rel_l2_mode", C.c_double),
                ("footprint_bytes", C.c_int64), ("t_arrival", C.c_double), ("t_admit", C.c_double),
                ("t_start", C.c_double), ("t_finish", C.c_double)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status"] = ERRORS.get(self.status, self.status)
        return d


_lib = None


def lib() -> C.CDLL:
    """Load the in-tree libdgw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1304_5546_amd.build`")
        # PyTorch ships its own HIP runtime under the same soname.  Load it
        # first so that libdgw.so binds to that one instance: one runtime per
        # process, so torch streams and device pointers are valid in the
        # library (two runtimes in one process do not share the device).
        if os.environ.get("DGW_NO_TORCH") != "1":
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "dgw_strerror": (C.c_char_p, [C.c_int]),
            "dgw_last_error": (C.c_char_p, []),
            "dgw_opts_default": (C.c_int, [P]),
            "dgw_reference_element": (C.c_int, [I32, I32, P, P, P, P, P, P, P, P, P, P, P]),
            "dgw_create": (C.c_int, [P, I32, P, P]),
            "dgw_destroy": (None, [P]),
            "dgw_sizes": (C.c_int, [P, P, P, P]),
            "dgw_node_coords": (C.c_int, [P, P, P, P]),
            "dgw_cfl_dt": (C.c_int, [P, P]),
            "dgw_set_fields": (C.c_int, [P, P]),
            "dgw_get_fields": (C.c_int, [P, P]),
            "dgw_set_cavity_mode": (C.c_int, [P, P]),
            "dgw_advance_steps": (C.c_int, [P, I64, D]),
            "dgw_advance": (C.c_int, [P, D, D, P]),
            "dgw_rhs": (C.c_int, [P, P, P]),
            "dgw_energy": (C.c_int, [P, P]),
            "dgw_energy_noalloc": (C.c_int, [P, P, P]),
            "dgw_cavity_error": (C.c_int, [P, P, D, P]),
            "dgw_last_info": (C.c_int, [P, P]),
            "dgw_set_fields_dev": (C.c_int, [P, P, P]),
            "dgw_get_fields_dev": (C.c_int, [P, P, P]),
            "dgw_launch_steps": (C.c_int, [P, I64, D, P]),
            "dgw_stage_cost": (C.c_int, [P, P, P]),
            "dgw_autotune": (C.c_int, [P, I32, P]),
            "dgw_footprint": (C.c_int, [P, I32, P, P]),
            "dgw_server_create": (C.c_int, [P, P]),
            "dgw_submit": (C.c_int, [P, P, P]),
            "dgw_poll": (C.c_int, [P, C.c_uint64, P]),
            "dgw_wait": (C.c_int, [P, C.c_uint64, P, P]),
            "dgw_cancel": (C.c_int, [P, C.c_uint64]),
            "dgw_server_stats": (C.c_int, [P, P, P, P]),
            "dgw_server_destroy": (None, [P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != 0:
        raise DgwError(rc, where, lib().dgw_last_error().decode())


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def reference_element(dim: int, order: int) -> dict:
    """The library's reference element (host FP64): nodes, Dr/Ds/Dt, M, LIFT,
    face node lists."""
    L = lib()
    Np, Nfp = C.c_int32(), C.c_int32()
    _check(L.dgw_reference_element(dim, order, C.byref(Np), C.byref(Nfp), *([None] * 9)), "dgw_reference_element")
    n, nf = Np.value, Nfp.value
    nfaces = dim + 1
    out = {k: np.zeros(n) for k in ("r", "s", "t")}
    for k in ("Dr", "Ds", "Dt", "M"):
        out[k] = np.zeros((n, n))
    out["LIFT"] = np.zeros((n, nfaces * nf))
    out["face_nodes"] = np.zeros((nfaces, nf), dtype=np.int32)
    _check(L.dgw_reference_element(dim, order, None, None, _ptr(out["r"]), _ptr(out["s"]), _ptr(out["t"]),
                                   _ptr(out["Dr"]), _ptr(out["Ds"]), _ptr(out["Dt"]), _ptr(out["M"]),
                                   _ptr(out["LIFT"]), _ptr(out["face_nodes"])), "dgw_reference_element")
    out["Np"], out["Nfp"] = n, nf
    return out


def default_opts(**kw) -> Opts:
    o = Opts()
    _check(lib().dgw_opts_default(C.byref(o)), "dgw_opts_default")
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PRECISIONS[v]
        setattr(o, k, v)
    return o


class Solver:
    """One DG Maxwell solve (2D TM or 3D) on the GPU behind the C ABI."""

    def __init__(self, mesh, order: int, *, alpha: float = 1.0, cfl: float = 1.0, prec="fp32",
                 renumber: bool = True, device: int = 0, stream=None, kernel: int = 0, lane_elems: int = 0,
                 wave_private: int = 0):
        L = lib()
        self._keep = []
        vx = np.ascontiguousarray(mesh.vx, dtype=np.float64)
        vy = np.ascontiguousarray(mesh.vy, dtype=np.float64)
        vz = None if mesh.vz is None else np.ascontiguousarray(mesh.vz, dtype=np.float64)
        ev = np.ascontiguousarray(mesh.elem_verts, dtype=np.int32)
        eps = None if mesh.eps is None else np.ascontiguousarray(mesh.eps, dtype=np.float64)
        mu = None if mesh.mu is None else np.ascontiguousarray(mesh.mu, dtype=np.float64)
        self._keep += [vx, vy, vz, ev, eps, mu]
        m = Mesh(mesh.dim, vx.size, _ptr(vx), _ptr(vy), _ptr(vz), ev.shape[0], _ptr(ev), _ptr(eps), _ptr(mu))
        o = default_opts(alpha=alpha, cfl=cfl, prec=prec, renumber=int(renumber), device=device, kernel=kernel,
                         lane_elems=lane_elems, wave_private=wave_private)
        if stream is not None:
            o.hip_stream = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        h = C.c_void_p()
        _check(L.dgw_create(C.byref(m), order, C.byref(o), C.byref(h)), "dgw_create")
        self._h = h
        K, Np, nf = C.c_int64(), C.c_int32(), C.c_int32()
        _check(L.dgw_sizes(h, C.byref(K), C.byref(Np), C.byref(nf)), "dgw_sizes")
        self.K, self.Np, self.n_fields = K.value, Np.value, nf.value
        self.dim = mesh.dim
        self.order = order

    def close(self):
        if getattr(self, "_h", None):
            lib().dgw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def shape(self):
        return (self.n_fields, self.K, self.Np)

    def node_coords(self):
        xs = [np.zeros((self.K, self.Np)) for _ in range(3)]
        _check(lib().dgw_node_coords(self._h, _ptr(xs[0]), _ptr(xs[1]), _ptr(xs[2]) if self.dim == 3 else None),
               "dgw_node_coords")
        return tuple(xs[: self.dim])

    def cfl_dt(self) -> float:
        d = C.c_double()
        _check(lib().dgw_cfl_dt(self._h, C.byref(d)), "dgw_cfl_dt")
        return d.value

    def set_fields(self, q: np.ndarray):
        q = np.ascontiguousarray(q, dtype=np.float64)
        if q.shape != self.shape:
            raise ValueError(f"fields must have shape {self.shape}")
        _check(lib().dgw_set_fields(self._h, _ptr(q)), "dgw_set_fields")

    def get_fields(self) -> np.ndarray:
        q = np.zeros(self.shape)
        _check(lib().dgw_get_fields(self._h, _ptr(q)), "dgw_get_fields")
        return q

    def set_cavity_mode(self, m: int, n: int, l: int = 0):
        mode = (C.c_int32 * 3)(m, n, l)
        _check(lib().dgw_set_cavity_mode(self._h, mode), "dgw_set_cavity_mode")

    def advance_steps(self, nsteps: int, dt: float = 0.0):
        _check(lib().dgw_advance_steps(self._h, int(nsteps), float(dt)), "dgw_advance_steps")

    def advance(self, t_final: float, dt: float = 0.0) -> int:
        n = C.c_int64()
        _check(lib().dgw_advance(self._h, float(t_final), float(dt), C.byref(n)), "dgw_advance")
        return n.value

    def rhs(self, q: np.ndarray) -> np.ndarray:
        q = np.ascontiguousarray(q, dtype=np.float64)
        if q.shape != self.shape:
            raise ValueError(f"fields must have shape {self.shape}")
        out = np.zeros(self.shape)
        _check(lib().dgw_rhs(self._h, _ptr(q), _ptr(out)), "dgw_rhs")
        return out

    def energy(self) -> float:
        e = C.c_double()
        _check(lib().dgw_energy(self._h, C.byref(e)), "dgw_energy")
        return e.value

    def energy_noalloc(self, out_tensor, stream=None):
        """dgw_energy_noalloc: the energy written asynchronously to a one-element
        FP64 device tensor on `stream` (None: the solver's stream)."""
        _check(lib().dgw_energy_noalloc(self._h, C.c_void_p(out_tensor.data_ptr()), self._stream_ptr(stream)),
               "dgw_energy_noalloc")

    def cavity_error(self, m: int, n: int, l: int, t: float) -> float:
        mode = (C.c_int32 * 3)(m, n, l)
        e = C.c_double()
        _check(lib().dgw_cavity_error(self._h, mode, float(t), C.byref(e)), "dgw_cavity_error")
        return e.value

    def info(self) -> dict:
        i = Info()
        _check(lib().dgw_last_info(self._h, C.byref(i)), "dgw_last_info")
        return {k: getattr(i, k) for k, _ in Info._fields_}

    def autotune(self, stages: int = 10) -> dict:
        """Time every kernel variant and launch shape that serves this solve
        (dgw_autotune) and keep the fastest; returns the choice and the
        timings of all candidates."""
        t = TuneInfo()
        _check(lib().dgw_autotune(self._h, int(stages), C.byref(t)), "dgw_autotune")
        n = t.n_tried
        return {"kernel": t.kernel, "groups_per_cu": t.groups_per_cu, "lane_elems": t.lane_elems,
                "wave_private": t.wave_private, "best_us": t.best_us,
                "tried": [{"kernel": t.tried_kernel[i], "groups_per_cu": t.tried_groups_per_cu[i],
                           "lane_elems": t.tried_lane_elems[i], "wave_private": t.tried_wave_private[i],
                           "us": t.tried_us[i]} for i in range(n)]}

    def stage_cost(self) -> tuple[float, float]:
        b, f = C.c_double(), C.c_double()
        _check(lib().dgw_stage_cost(self._h, C.byref(b), C.byref(f)), "dgw_stage_cost")
        return b.value, f.value

    # --- device-pointer plumbing (torch tensors / streams) -----------------
    @staticmethod
    def _stream_ptr(stream):
        if stream is None:
            return None
        return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))

    def set_fields_dev(self, q_tensor, stream=None):
        if tuple(q_tensor.shape) != self.shape or not q_tensor.is_contiguous() or str(q_tensor.dtype) != "torch.float32":
            raise ValueError(f"need a contiguous float32 device tensor of shape {self.shape}")
        _check(lib().dgw_set_fields_dev(self._h, C.c_void_p(q_tensor.data_ptr()), self._stream_ptr(stream)),
               "dgw_set_fields_dev")

    def get_fields_dev(self, q_tensor, stream=None):
        if tuple(q_tensor.shape) != self.shape or not q_tensor.is_contiguous() or str(q_tensor.dtype) != "torch.float32":
            raise ValueError(f"need a contiguous float32 device tensor of shape {self.shape}")
        _check(lib().dgw_get_fields_dev(self._h, C.c_void_p(q_tensor.data_ptr()), self._stream_ptr(stream)),
               "dgw_get_fields_dev")

    def launch_steps(self, nsteps: int, dt: float, stream=None):
        _check(lib().dgw_launch_steps(self._h, int(nsteps), float(dt), self._stream_ptr(stream)), "dgw_launch_steps")


def _mesh_struct(mesh, keep: list) -> Mesh:
    vx = np.ascontiguousarray(mesh.vx, dtype=np.float64)
    vy = np.ascontiguousarray(mesh.vy, dtype=np.float64)
    vz = None if mesh.vz is None else np.ascontiguousarray(mesh.vz, dtype=np.float64)
    ev = np.ascontiguousarray(mesh.elem_verts, dtype=np.int32)
    eps = None if mesh.eps is None else np.ascontiguousarray(mesh.eps, dtype=np.float64)
    mu = None if mesh.mu is None else np.ascontiguousarray(mesh.mu, dtype=np.float64)
    keep += [vx, vy, vz, ev, eps, mu]
    return Mesh(mesh.dim, vx.size, _ptr(vx), _ptr(vy), _ptr(vz), ev.shape[0], _ptr(ev), _ptr(eps), _ptr(mu))


def footprint(mesh, order: int, prec="fp32") -> int:
    """Device bytes a solver of this mesh and order allocates."""
    keep: list = []
    m = _mesh_struct(mesh, keep)
    o = default_opts(prec=prec)
    b = C.c_int64()
    _check(lib().dgw_footprint(C.byref(m), order, C.byref(o), C.byref(b)), "dgw_footprint")
    return b.value


class Server:
    """Continuous-batching request server (``dgw_server_*``): submit cavity
    solves, wait for their results."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 0, device: int = 0, setup_threads: int = 0,
                 max_chunk_steps: int = 0):
        o = ServerOpts(hbm_budget_bytes, max_slots, device, setup_threads, max_chunk_steps)
        h = C.c_void_p()
        _check(lib().dgw_server_create(C.byref(o), C.byref(h)), "dgw_server_create")
        self._h = h
        self._np = {}

    def submit(self, mesh, order: int, *, mode=(1, 1), q0: np.ndarray | None = None, t_final: float = 1.0,
               alpha: float = 1.0, prec="fp32", keep_fields: bool = False) -> int:
        keep: list = []
        m = _mesh_struct(mesh, keep)
        q = None if q0 is None else np.ascontiguousarray(q0, dtype=np.float64)
        md = (C.c_int32 * 3)(*(list(mode) + [0] * (3 - len(mode))))
        r = Request(m, order, md, _ptr(q), t_final, alpha, PRECISIONS[prec] if isinstance(prec, str) else prec,
                    int(keep_fields))
        t = C.c_uint64()
        _check(lib().dgw_submit(self._h, C.byref(r), C.byref(t)), "dgw_submit")
        self._np[t.value] = (mesh.elem_verts.shape[0], (order + 1) * (order + 2) // 2)
        return t.value

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        _check(lib().dgw_poll(self._h, ticket, C.byref(d)), "dgw_poll")
        return bool(d.value)

    def wait(self, ticket: int, fields: bool = False):
        """Block until the request ends; returns (result dict, fields or None).
        A cancelled request returns status DGW_ECANCELLED (no exception)."""
        K, Np = self._np.get(ticket, (0, 0))
        q = np.zeros((3, K, Np)) if fields else None
        res = Result()
        rc = lib().dgw_wait(self._h, ticket, _ptr(q), C.byref(res))
        if rc not in (0, -8) and res.status == 0:
            _check(rc, "dgw_wait")
        self._np.pop(ticket, None)
        return res.as_dict(), (q if rc == 0 else None)

    def cancel(self, ticket: int):
        _check(lib().dgw_cancel(self._h, ticket), "dgw_cancel")

    def stats(self) -> dict:
        n, d, b = C.c_int64(), C.c_double(), C.c_double()
        _check(lib().dgw_server_stats(self._h, C.byref(n), C.byref(d), C.byref(b)), "dgw_server_stats")
        return {"completed": n.value, "dof_updates": d.value, "busy_s": b.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().dgw_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
