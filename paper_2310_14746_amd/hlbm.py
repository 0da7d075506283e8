"""Thin ctypes binding of the C-ABI in ``include/hlbm.h`` (``libhlbm.so``).

Only argument marshalling lives here: every step of the sweep runs in the HIP
kernels of the library.  PyTorch supplies device memory (population buffers and
the porosity field are torch tensors bound with ``hlbm_bind_buffers``) and the
stream (torch's current stream).  If the library has not been built, loading
fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhlbm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hlbm.h")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5, -6
BATCH_GRAPH, BATCH_PERSISTENT, BATCH_PER_STEP, BATCH_GRAPH_PERSISTENT = 0, 1, 2, 3
BATCH_MODES = {"graph": BATCH_GRAPH, "persistent": BATCH_PERSISTENT, "per_step": BATCH_PER_STEP,
               "graph_persistent": BATCH_GRAPH_PERSISTENT}
D2Q9, D3Q19 = 9, 19
F64, F32, F16S, BF16S = 0, 1, 2, 3
AB, AA = 0, 1
PATTERNS = {"ab": AB, "aa": AA}
PERIODIC, WALL, INLET_U, OUTLET_RHO = 0, 1, 2, 3
POROSITY_SCALAR, POROSITY_TENSOR = 0, 1
TAPE_REPLAY, TAPE_MOMENTS = 0, 1
POROSITY_KINDS = {"scalar": POROSITY_SCALAR, "tensor": POROSITY_TENSOR}
DT_F64, DT_F32, DT_F16 = 0, 1, 2

STORAGE = {"f64": F64, "f32": F32, "f16s": F16S, "bf16s": BF16S}
_STORE_ELEM = {F64: 8, F32: 4, F16S: 2, BF16S: 2}
_POROSITY_DTYPE = {F64: "f64", F32: "f32", F16S: "f16", BF16S: "f16"}


class HLBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hlbm error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("storage", ctypes.c_int),
        ("pattern", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("bc_lo", ctypes.c_int * 3),
        ("bc_hi", ctypes.c_int * 3),
        ("inlet_u", ctypes.c_double * 3),
        ("outlet_rho", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("store_scale", ctypes.c_double),
        ("external_memory", ctypes.c_int),
        ("block_x", ctypes.c_int),
        ("hip_stream", ctypes.c_void_p),
        ("porosity_kind", ctypes.c_int),
        ("row_pad_bytes", ctypes.c_int),
    ]


_lib = None


def declared_functions() -> list:
    """Names of the functions declared in the headers under include/ (hlbm.h
    and the bandwidth reference beside it)."""
    names = []
    inc = os.path.dirname(HEADER)
    for h in sorted(os.listdir(inc)):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(inc, h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(hlbm_\w+)\s*\(", text, flags=re.M)
    return names


def load() -> ctypes.CDLL:
    """Load libhlbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime; import it first so that libhlbm.so binds
    # to that same runtime (one runtime per process: the library and torch
    # exchange device pointers and streams).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2310_14746_amd.build` "
            "(the HIP library is the only compute path)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "hlbm_version": ([], i),
        "hlbm_last_error": ([], ctypes.c_char_p),
        "hlbm_config_default": ([P(Config)], i),
        "hlbm_lattice_info": ([i, P(ctypes.c_int), P(ctypes.c_double)], i),
        "hlbm_required_bytes": ([P(Config), P(ctypes.c_size_t), P(ctypes.c_size_t)], i),
        "hlbm_create": ([P(Config), P(vp)], i),
        "hlbm_bind_buffers": ([vp, vp, vp, vp], i),
        "hlbm_destroy": ([vp], i),
        "hlbm_set_porosity": ([vp, vp, i, i], i),
        "hlbm_step": ([vp, i], i),
        "hlbm_get_step": ([vp, P(ctypes.c_longlong)], i),
        "hlbm_moments": ([vp, vp, vp, i, i, P(ctypes.c_double)], i),
        "hlbm_moments_noalloc": ([vp, vp, vp, i, vp], i),
        "hlbm_state_bytes": ([vp, P(ctypes.c_size_t)], i),
        "hlbm_get_state": ([vp, vp, i, P(ctypes.c_longlong)], i),
        "hlbm_set_state": ([vp, vp, i, ctypes.c_longlong], i),
        "hlbm_reset": ([vp], i),
        "hlbm_sync": ([vp], i),
        "hlbm_create_batch": ([P(Config), i, P(vp)], i),
        "hlbm_batch_info": ([vp, P(ctypes.c_int), P(ctypes.c_size_t)], i),
        "hlbm_batch_set_mode": ([vp, i], i),
        "hlbm_batch_set_schedule": ([vp, i, i], i),
        "hlbm_batch_set_barrier_limit": ([vp, i], i),
        "hlbm_batch_get_schedule": ([vp, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int)], i),
        "hlbm_batch_set_porosity": ([vp, i, vp, i, i], i),
        "hlbm_batch_moments": ([vp, i, vp, vp, i, P(ctypes.c_double)], i),
        "hlbm_batch_set_solid_mask": ([vp, i, vp, i], i),
        "hlbm_set_solid_mask": ([vp, vp, i], i),
        "hlbm_set_diagnostics": ([vp, i, i], i),
        "hlbm_read_diagnostics": ([vp, P(ctypes.c_double), i, P(ctypes.c_int), P(ctypes.c_longlong)], i),
        "hlbm_set_tape": ([vp, i, i], i),
        "hlbm_set_tape_kind": ([vp, i], i),
        "hlbm_tape_info": ([vp, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_longlong),
                            P(ctypes.c_size_t)], i),
        "hlbm_adjoint_step": ([vp, i, vp, vp, vp, i], i),
        "hlbm_ref_stream_pattern": ([vp, vp, vp, i, i, i, i, i, vp], i),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        msg = load().hlbm_last_error()
        raise HLBMError(rc, msg.decode() if msg else "")


def lattice_info(q: int):
    """(c[q,3], w[q]) in the library's population order."""
    c = (ctypes.c_int * (3 * q))()
    w = (ctypes.c_double * q)()
    _check(load().hlbm_lattice_info(q, c, w))
    return np.array(c, dtype=np.int64).reshape(q, 3), np.array(w)


def make_config(lattice: int = D3Q19, storage="f32", shape=(32, 32, 32), tau: float = 0.6,
                force=(0.0, 0.0, 0.0), bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), inlet_u=(0.0, 0.0, 0.0),
                outlet_rho: float = 1.0, rho0: float = 1.0, store_scale: float = 1.0,
                block_x: int = 0, external_memory: int = 0, stream: Optional[int] = None,
                porosity: str = "scalar", pattern: str = "ab", row_pad: int = 0) -> Config:
    cfg = Config()
    _check(load().hlbm_config_default(ctypes.byref(cfg)))
    cfg.lattice = int(lattice)
    cfg.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    cfg.pattern = PATTERNS[pattern]
    nx, ny, nz = (tuple(shape) + (1,))[:3] if len(shape) == 2 else tuple(shape)
    cfg.nx, cfg.ny, cfg.nz = int(nx), int(ny), int(nz)
    cfg.tau = float(tau)
    cfg.force = (ctypes.c_double * 3)(*[float(v) for v in force])
    cfg.bc_lo = (ctypes.c_int * 3)(*[int(v) for v in bc_lo])
    cfg.bc_hi = (ctypes.c_int * 3)(*[int(v) for v in bc_hi])
    cfg.inlet_u = (ctypes.c_double * 3)(*[float(v) for v in inlet_u])
    cfg.outlet_rho = float(outlet_rho)
    cfg.rho0 = float(rho0)
    cfg.store_scale = float(store_scale)
    cfg.block_x = int(block_x)
    cfg.external_memory = int(external_memory)
    cfg.hip_stream = stream
    cfg.porosity_kind = POROSITY_KINDS[porosity]
    cfg.row_pad_bytes = int(row_pad)
    return cfg


class HLBM:
    """One lattice (context).  Device memory comes from torch tensors.

    ``shape`` is (nx, ny, nz); fields returned by :meth:`moments` have shape
    (nz, ny, nx) for drho and (3, nz, ny, nx) for u.  ``pattern`` "ab" keeps two
    population buffers; "aa" updates one in place (periodic and wall faces).
    ``row_pad`` pads every population row by that many bytes (a multiple of
    256; :func:`tune.lookup_row_pad` gives the measured choice for a shape).
    """

    def __init__(self, lattice: int = D3Q19, storage="f32", shape=(32, 32, 32), tau=0.6,
                 force=(0.0, 0.0, 0.0), bc_lo=(0, 0, 0), bc_hi=(0, 0, 0),
                 inlet_u=(0.0, 0.0, 0.0), outlet_rho=1.0, rho0=1.0, store_scale=1.0,
                 block_x=0, device="cuda:0", porosity="scalar", pattern="ab", row_pad=0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        lib = load()
        self.cfg = make_config(lattice, storage, shape, tau, force, bc_lo, bc_hi, inlet_u,
                               outlet_rho, rho0, store_scale, block_x, external_memory=1,
                               stream=self.stream.cuda_stream, porosity=porosity, pattern=pattern,
                               row_pad=row_pad)
        self.pattern = pattern
        self.q = self.cfg.lattice
        self.porosity_rows = 6 if porosity == "tensor" else 1
        self.storage = self.cfg.storage
        self.shape = (self.cfg.nx, self.cfg.ny, self.cfg.nz)
        self.N = self.cfg.nx * self.cfg.ny * self.cfg.nz
        pb, db = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib.hlbm_required_bytes(ctypes.byref(self.cfg), ctypes.byref(pb), ctypes.byref(db)))
        self.pop_bytes = pb.value
        with torch.cuda.device(self.device):
            self._pop_a = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
            # the in-place pattern keeps one population buffer
            self._pop_b = (None if pattern == "aa"
                           else torch.empty(pb.value, dtype=torch.uint8, device=self.device))
            self._dfield = torch.empty(max(db.value, 1), dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        _check(lib.hlbm_create(ctypes.byref(self.cfg), ctypes.byref(ctx)))
        self.ctx = ctx
        # bumped by every call that changes the state, the control or the tape:
        # a gradient taken from a tape is valid only at the generation it was
        # recorded in
        self.generation = 0
        _check(lib.hlbm_bind_buffers(self.ctx, self._pop_a.data_ptr(),
                                     None if self._pop_b is None else self._pop_b.data_ptr(),
                                     self._dfield.data_ptr()))

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            rc = load().hlbm_destroy(self.ctx)
            self.ctx = None
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- porosity ----------------------------------------------------------
    def set_porosity(self, d):
        """d = 1 - varpi per cell (or, for porosity="tensor", rows xx, yy, zz, xy,
        xz, yz of D, shape (6, N)): numpy array (host) or torch tensor (host or
        device)."""
        self.generation += 1
        t = self.torch
        if isinstance(d, t.Tensor):
            dd = d.contiguous()
            dtype = {t.float64: DT_F64, t.float32: DT_F32, t.float16: DT_F16}[dd.dtype]
            if dd.numel() != self.N * self.porosity_rows:
                raise ValueError(f"porosity needs {self.porosity_rows} x nx*ny*nz values")
            on_dev = 1 if dd.is_cuda else 0
            if on_dev:
                _check(load().hlbm_set_porosity(self.ctx, dd.data_ptr(), dtype, 1))
            else:
                arr = dd.numpy()
                _check(load().hlbm_set_porosity(self.ctx, arr.ctypes.data, dtype, 0))
            return
        arr = np.ascontiguousarray(d)
        if arr.size != self.N * self.porosity_rows:
            raise ValueError(f"porosity needs {self.porosity_rows} x nx*ny*nz values")
        dtype = {np.dtype(np.float64): DT_F64, np.dtype(np.float32): DT_F32,
                 np.dtype(np.float16): DT_F16}[arr.dtype]
        _check(load().hlbm_set_porosity(self.ctx, arr.ctypes.data, dtype, 0))

    @property
    def porosity_dtype(self) -> str:
        return _POROSITY_DTYPE[self.storage]

    # -- stepping ----------------------------------------------------------
    def step(self, n: int = 1):
        self.generation += 1
        _check(load().hlbm_step(self.ctx, int(n)))

    @property
    def step_count(self) -> int:
        s = ctypes.c_longlong()
        _check(load().hlbm_get_step(self.ctx, ctypes.byref(s)))
        return s.value

    def sync(self):
        _check(load().hlbm_sync(self.ctx))

    def reset(self):
        self.generation += 1
        _check(load().hlbm_reset(self.ctx))

    # -- observation -------------------------------------------------------
    def moments(self, dtype: str = "f64", device: bool = True, totals: bool = False):
        """(drho, u[, totals]) at the current time level as torch tensors."""
        t = self.torch
        tdt = t.float64 if dtype == "f64" else t.float32
        cdt = DT_F64 if dtype == "f64" else DT_F32
        nx, ny, nz = self.shape
        tot = (ctypes.c_double * 4)()
        if device:
            drho = t.empty((nz, ny, nx), dtype=tdt, device=self.device)
            u = t.empty((3, nz, ny, nx), dtype=tdt, device=self.device)
            _check(load().hlbm_moments(self.ctx, drho.data_ptr(), u.data_ptr(), cdt, 1, tot))
        else:
            drho = t.empty((nz, ny, nx), dtype=tdt)
            u = t.empty((3, nz, ny, nx), dtype=tdt)
            _check(load().hlbm_moments(self.ctx, drho.data_ptr(), u.data_ptr(), cdt, 0, tot))
        if totals:
            return drho, u, np.array(tot)
        return drho, u

    def totals(self) -> np.ndarray:
        """FP64 [sum(rho - rho0), sum rho u_x, sum rho u_y, sum rho u_z] over fluid cells."""
        tot = (ctypes.c_double * 4)()
        _check(load().hlbm_moments(self.ctx, None, None, DT_F64, 1, tot))
        return np.array(tot)

    def moments_noalloc(self, drho=None, u=None, totals=None):
        """Enqueue hlbm_moments_noalloc into caller-owned device tensors (drho
        (nz, ny, nx) and u (3, nz, ny, nx), both f64 or both f32; totals 4 f64);
        nothing is allocated or awaited."""
        t = self.torch
        ref = drho if drho is not None else u
        cdt = DT_F32 if ref is not None and ref.dtype == t.float32 else DT_F64
        for a in (drho, u, totals):
            if a is not None and not (a.is_cuda and a.is_contiguous()):
                raise ValueError("moments_noalloc writes contiguous device tensors")
        if totals is not None and (totals.dtype != t.float64 or totals.numel() < 4):
            raise ValueError("totals must hold 4 float64 values")
        ptr = (lambda a: None if a is None else a.data_ptr())
        _check(load().hlbm_moments_noalloc(self.ctx, ptr(drho), ptr(u), cdt, ptr(totals)))

    # -- state -------------------------------------------------------------
    @property
    def state_bytes(self) -> int:
        """Bytes of one snapshot: q rows of N stored values (the population
        buffers themselves pad their rows, see pop_bytes)."""
        nb = ctypes.c_size_t()
        _check(load().hlbm_state_bytes(self.ctx, ctypes.byref(nb)))
        return nb.value

    def get_state(self):
        """(raw state bytes as a uint8 device tensor, step)."""
        t = self.torch
        buf = t.empty(self.state_bytes, dtype=t.uint8, device=self.device)
        s = ctypes.c_longlong()
        _check(load().hlbm_get_state(self.ctx, buf.data_ptr(), 1, ctypes.byref(s)))
        return buf, s.value

    def set_state(self, buf, step: int):
        self.generation += 1
        if buf.numel() != self.state_bytes:
            raise ValueError("state size mismatch")
        _check(load().hlbm_set_state(self.ctx, buf.contiguous().data_ptr(), 1 if buf.is_cuda else 0,
                                     int(step)))

    # -- resolved obstacles ------------------------------------------------
    def set_solid_mask(self, mask):
        """Solid cells (nonzero) of a periodic box, shape (nz, ny, nx) or N; None removes them."""
        self.generation += 1
        if mask is None:
            _check(load().hlbm_set_solid_mask(self.ctx, None, 0))
            return
        t = self.torch
        if isinstance(mask, t.Tensor):
            m = mask.reshape(-1).to(t.uint8).contiguous()
            if m.numel() != self.N:
                raise ValueError("mask needs nx*ny*nz values")
            _check(load().hlbm_set_solid_mask(self.ctx, m.data_ptr(), 1 if m.is_cuda else 0))
            return
        m = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
        if m.size != self.N:
            raise ValueError("mask needs nx*ny*nz values")
        _check(load().hlbm_set_solid_mask(self.ctx, m.ctypes.data, 0))

    # -- in-sweep diagnostics ------------------------------------------------
    def set_diagnostics(self, every: int, capacity: int = 1024):
        """Record FP64 totals inside the sweep at time levels n % every == 0."""
        _check(load().hlbm_set_diagnostics(self.ctx, int(every), int(capacity)))

    def read_diagnostics(self, max_records: int = 1 << 20):
        """(steps[k], totals[k, 4], dropped) of the records since the last read."""
        cap = max(1, int(max_records))
        buf = (ctypes.c_double * (5 * cap))()
        n, dropped = ctypes.c_int(), ctypes.c_longlong()
        _check(load().hlbm_read_diagnostics(self.ctx, buf, cap, ctypes.byref(n), ctypes.byref(dropped)))
        arr = np.frombuffer(buf, dtype=np.float64)[:5 * n.value].reshape(n.value, 5).copy()
        return arr[:, 0].astype(np.int64), arr[:, 1:], dropped.value

    # -- adjoint -----------------------------------------------------------
    def set_tape(self, every: int, max_steps: int):
        """Record checkpoints every `every` steps for up to `max_steps` steps from now."""
        self.generation += 1
        _check(load().hlbm_set_tape(self.ctx, int(every), int(max_steps)))

    def set_tape_kind(self, kind: str):
        """"replay" (checkpoints, segments replayed in the reverse sweep) or
        "moments" (every recorded step also keeps each cell's FP64 moments, so
        the reverse sweep replays nothing)."""
        self.generation += 1
        _check(load().hlbm_set_tape_kind(self.ctx, {"replay": TAPE_REPLAY, "moments": TAPE_MOMENTS}[kind]))

    def tape_info(self) -> dict:
        e, m, r, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong(), ctypes.c_size_t()
        _check(load().hlbm_tape_info(self.ctx, ctypes.byref(e), ctypes.byref(m), ctypes.byref(r),
                                     ctypes.byref(b)))
        return {"every": e.value, "max_steps": m.value, "recorded": r.value,
                "device_bytes": b.value}

    def adjoint(self, nsteps: int, drho_bar, u_bar, d_bar=None):
        """Reverse sweep over the last `nsteps` recorded steps.

        drho_bar (N values) and u_bar (3*N values) are the cotangents of the
        current moments (shapes as returned by :meth:`moments`); returns d_bar
        (FP64 device tensor shaped (nz, ny, nx), or (6, nz, ny, nx) for a
        tensor control: rows xx, yy, zz, xy, xz, yz) with dJ/dd through those
        steps added to `d_bar` if given (else to zeros).
        """
        t = self.torch
        nx, ny, nz = self.shape
        rows = self.porosity_rows
        gr = t.as_tensor(drho_bar, dtype=t.float64, device=self.device).contiguous()
        gu = t.as_tensor(u_bar, dtype=t.float64, device=self.device).contiguous()
        if gr.numel() != self.N or gu.numel() != 3 * self.N:
            raise ValueError("cotangents need N and 3*N values")
        if d_bar is None:
            d_bar = t.zeros(((rows,) if rows > 1 else ()) + (nz, ny, nx), dtype=t.float64, device=self.device)
        elif not (d_bar.dtype == t.float64 and d_bar.is_cuda and d_bar.is_contiguous()
                  and d_bar.numel() == rows * self.N):
            raise ValueError(f"d_bar must be a contiguous FP64 device tensor of {rows}*N values")
        _check(load().hlbm_adjoint_step(self.ctx, int(nsteps), gr.data_ptr(), gu.data_ptr(),
                                        d_bar.data_ptr(), 1))
        return d_bar

    def state_f64(self, store_scale: Optional[float] = None) -> np.ndarray:
        """Current post-collision populations as float64 g[i, cell] (library order)."""
        t = self.torch
        buf, _ = self.get_state()
        raw = buf.cpu()
        if self.storage == F64:
            v = raw.view(t.float64).numpy().astype(np.float64)
        elif self.storage == F32:
            v = raw.view(t.float32).numpy().astype(np.float64)
        elif self.storage == F16S:
            v = raw.view(t.float16).to(t.float64).numpy() / self.cfg.store_scale
        else:
            v = raw.view(t.bfloat16).to(t.float64).numpy() / self.cfg.store_scale
        return v.reshape(self.q, self.N)


def _host_or_device(d, n, torch):
    """(pointer, dtype code, on_device, keepalive) for a porosity array."""
    if isinstance(d, torch.Tensor):
        dd = d.contiguous()
        if dd.numel() != n:
            raise ValueError(f"porosity needs {n} values")
        code = {torch.float64: DT_F64, torch.float32: DT_F32, torch.float16: DT_F16}[dd.dtype]
        if dd.is_cuda:
            return dd.data_ptr(), code, 1, dd
        arr = dd.numpy()
        return arr.ctypes.data, code, 0, arr
    arr = np.ascontiguousarray(d)
    if arr.size != n:
        raise ValueError(f"porosity needs {n} values")
    code = {np.dtype(np.float64): DT_F64, np.dtype(np.float32): DT_F32,
            np.dtype(np.float16): DT_F16}[arr.dtype]
    return arr.ctypes.data, code, 0, arr


class HLBMBatch:
    """Many independent periodic D3Q19 boxes advanced together.

    ``items`` is a sequence of dicts with keys ``shape`` (nx, ny, nz), ``tau``
    and ``force``.  The library owns the packed device memory; torch supplies
    the stream.  ``tile`` (cells per tile = threads per block, 0 = 256),
    ``blocks_per_cu`` and ``chunk`` (0 = defaults) set the persistent kernel's
    schedule, ``row_pad`` the padding in bytes after each packed population
    row; results depend on neither.
    """

    def __init__(self, items, storage="f32", store_scale=1.0, rho0=1.0, mode="graph",
                 device="cuda:0", tile=0, blocks_per_cu=0, chunk=0, row_pad=0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        lib = load()
        n = len(items)
        arr = (Config * n)()
        for k, it in enumerate(items):
            c = make_config(D3Q19, storage, it["shape"], it["tau"], it.get("force", (0, 0, 0)),
                            rho0=rho0, store_scale=store_scale, stream=self.stream.cuda_stream,
                            block_x=tile if k == 0 else 0, row_pad=row_pad if k == 0 else 0)
            arr[k] = c
        self.items = [dict(shape=tuple(int(v) for v in it["shape"]), tau=float(it["tau"]),
                           force=tuple(float(v) for v in it.get("force", (0, 0, 0))))
                      for it in items]
        ctx = ctypes.c_void_p()
        _check(lib.hlbm_create_batch(arr, n, ctypes.byref(ctx)))
        self.ctx = ctx
        self.n_items = n
        self.set_mode(mode)
        if blocks_per_cu or chunk:
            self.set_schedule(blocks_per_cu, chunk)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            rc = load().hlbm_destroy(self.ctx)
            self.ctx = None
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def info(self):
        n, cells = ctypes.c_int(), ctypes.c_size_t()
        _check(load().hlbm_batch_info(self.ctx, ctypes.byref(n), ctypes.byref(cells)))
        return n.value, cells.value

    def set_mode(self, mode):
        _check(load().hlbm_batch_set_mode(self.ctx, BATCH_MODES[mode] if isinstance(mode, str)
                                          else int(mode)))

    def set_schedule(self, blocks_per_cu: int = 0, chunk: int = 0):
        """Resident blocks per CU and tiles per draw of the persistent kernel (0 = default)."""
        _check(load().hlbm_batch_set_schedule(self.ctx, int(blocks_per_cu), int(chunk)))

    def set_barrier_limit(self, polls: int):
        """Bound on the persistent kernel's barrier wait (polls of ~0.1 us)."""
        _check(load().hlbm_batch_set_barrier_limit(self.ctx, int(polls)))

    def schedule(self) -> dict:
        t, b, m, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().hlbm_batch_get_schedule(self.ctx, ctypes.byref(t), ctypes.byref(b), ctypes.byref(m),
                                              ctypes.byref(c)))
        return {"tile": t.value, "blocks_per_cu": b.value, "max_blocks_per_cu": m.value, "chunk": c.value}

    def set_porosity(self, item: int, d):
        nx, ny, nz = self.items[item]["shape"]
        ptr, code, on_dev, keep = _host_or_device(d, nx * ny * nz, self.torch)
        _check(load().hlbm_batch_set_porosity(self.ctx, int(item), ptr, code, on_dev))
        del keep

    def set_solid_mask(self, item: int, mask):
        """Resolved obstacles of one item: nonzero cells of `mask` (shape
        (nz, ny, nx) or nx*ny*nz) are solid; None removes them."""
        if mask is None:
            _check(load().hlbm_batch_set_solid_mask(self.ctx, int(item), None, 0))
            return
        nx, ny, nz = self.items[item]["shape"]
        t = self.torch
        if isinstance(mask, t.Tensor):
            m = mask.reshape(-1).to(t.uint8).contiguous()
            if m.numel() != nx * ny * nz:
                raise ValueError("mask needs nx*ny*nz values")
            _check(load().hlbm_batch_set_solid_mask(self.ctx, int(item), m.data_ptr(), 1 if m.is_cuda else 0))
            return
        m = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
        if m.size != nx * ny * nz:
            raise ValueError("mask needs nx*ny*nz values")
        _check(load().hlbm_batch_set_solid_mask(self.ctx, int(item), m.ctypes.data, 0))

    def step(self, n: int = 1):
        _check(load().hlbm_step(self.ctx, int(n)))

    def sync(self):
        _check(load().hlbm_sync(self.ctx))

    def reset(self):
        """Every item back to rest (g = 0) and step 0; the porosity is kept."""
        _check(load().hlbm_reset(self.ctx))

    @property
    def step_count(self) -> int:
        s = ctypes.c_longlong()
        _check(load().hlbm_get_step(self.ctx, ctypes.byref(s)))
        return s.value

    def moments(self, item: int):
        """(drho (nz,ny,nx), u (3,nz,ny,nx)) of one item, FP64 device tensors."""
        t = self.torch
        nx, ny, nz = self.items[item]["shape"]
        drho = t.empty((nz, ny, nx), dtype=t.float64, device=self.device)
        u = t.empty((3, nz, ny, nx), dtype=t.float64, device=self.device)
        _check(load().hlbm_batch_moments(self.ctx, int(item), drho.data_ptr(), u.data_ptr(), 1, None))
        return drho, u

    def totals(self) -> np.ndarray:
        """FP64 [sum(rho - rho0), sum rho u_x, sum rho u_y, sum rho u_z] per item."""
        tot = (ctypes.c_double * (4 * self.n_items))()
        _check(load().hlbm_batch_moments(self.ctx, -1, None, None, 1, tot))
        return np.array(tot).reshape(self.n_items, 4)

    def get_state(self):
        t = self.torch
        nb = ctypes.c_size_t()
        _check(load().hlbm_state_bytes(self.ctx, ctypes.byref(nb)))
        buf = t.empty(nb.value, dtype=t.uint8, device=self.device)
        s = ctypes.c_longlong()
        _check(load().hlbm_get_state(self.ctx, buf.data_ptr(), 1, ctypes.byref(s)))
        return buf, s.value
