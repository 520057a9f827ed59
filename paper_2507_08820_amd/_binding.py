"""ctypes binding of librflbm (include/rflbm.h): argument marshalling only.

Every computation runs in the HIP kernels of librflbm.so.  PyTorch provides
device memory (the lattice buffer and readback tensors) and the HIP stream.
If the library has not been built, loading fails with an ImportError instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RFLBM_LIBRARY") or os.path.join(_HERE, "librflbm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "rflbm.h")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
MODEL = {"reg": 0, "bgk": 1, "rec": 2}
M_RHO, M_J, M_PI = 1, 2, 4
FIELDS = ("rho", "jx", "jy", "jz", "pi_xx", "pi_yy", "pi_zz", "pi_xy", "pi_xz", "pi_yz")


class RFLBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rflbm status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("storage", ctypes.c_int32), ("model", ctypes.c_int32),
        ("philox_rounds", ctypes.c_uint32),
        ("rho0", ctypes.c_double), ("kT", ctypes.c_double),
        ("tau_shear", ctypes.c_double), ("tau_bulk", ctypes.c_double),
        ("tau_ghost", ctypes.c_double * 17),
        ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
        ("storage_scale", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("samples", ctypes.c_int64), ("nodes", ctypes.c_int64),
        ("sum_drho", ctypes.c_double), ("sum_drho2", ctypes.c_double),
        ("sum_j", ctypes.c_double * 3), ("sum_j2", ctypes.c_double * 3),
        ("sum_u2", ctypes.c_double * 3),
        ("sum_pi", ctypes.c_double * 6), ("sum_pi2", ctypes.c_double * 6),
        ("mass_dev", ctypes.c_double), ("momentum", ctypes.c_double * 3),
    ]

    def as_dict(self) -> dict:
        return {
            "samples": self.samples, "nodes": self.nodes,
            "sum_drho": self.sum_drho, "sum_drho2": self.sum_drho2,
            "sum_j": np.array(self.sum_j[:]), "sum_j2": np.array(self.sum_j2[:]),
            "sum_u2": np.array(self.sum_u2[:]),
            "sum_pi": np.array(self.sum_pi[:]), "sum_pi2": np.array(self.sum_pi2[:]),
            "mass_dev": self.mass_dev, "momentum": np.array(self.momentum[:]),
        }


_lib = None

_VP = ctypes.c_void_p
_PP = ctypes.POINTER(Params)
_SIGS = {
    "rflbm_params_default": (None, [_PP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "rflbm_required_bytes": (ctypes.c_size_t, [_PP]),
    "rflbm_create": (ctypes.c_int, [_PP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "rflbm_destroy": (ctypes.c_int, [_VP]),
    "rflbm_set_params": (ctypes.c_int, [_VP, _PP]),
    "rflbm_get_params": (ctypes.c_int, [_VP, _PP]),
    "rflbm_init_equilibrium": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int]),
    "rflbm_init_thermal": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int]),
    "rflbm_step": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "rflbm_sync": (ctypes.c_int, [_VP]),
    "rflbm_step_count": (ctypes.c_int64, [_VP]),
    "rflbm_set_step_count": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "rflbm_get_populations": (ctypes.c_int, [_VP, _VP, ctypes.c_int]),
    "rflbm_set_populations": (ctypes.c_int, [_VP, _VP, ctypes.c_int]),
    "rflbm_get_populations_at": (ctypes.c_int, [_VP, _VP, ctypes.c_uint32, _VP]),
    "rflbm_get_moments": (ctypes.c_int, [_VP, ctypes.c_uint32, _VP, ctypes.c_int]),
    "rflbm_get_moments_host_noalloc": (ctypes.c_int, [_VP, ctypes.c_uint32, _VP]),
    "rflbm_stats_config": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "rflbm_get_stats": (ctypes.c_int, [_VP, ctypes.POINTER(Stats)]),
    "rflbm_reset_stats": (ctypes.c_int, [_VP]),
    "rflbm_sk_sample": (ctypes.c_int, [_VP]),
    "rflbm_sk_nshells": (ctypes.c_int32, [_VP]),
    "rflbm_get_sk": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int64)]),
    "rflbm_reset_sk": (ctypes.c_int, [_VP]),
    "rflbm_set_launch": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "rflbm_get_launch": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "rflbm_set_row_blocks": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "rflbm_get_row_blocks": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    "rflbm_time_steps": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "rflbm_batch_required_bytes": (ctypes.c_size_t, [ctypes.c_int32, _PP]),
    "rflbm_batch_create": (ctypes.c_int, [ctypes.c_int32, _PP, _VP, ctypes.c_size_t, _VP,
                                          ctypes.POINTER(_VP)]),
    "rflbm_batch_destroy": (ctypes.c_int, [_VP]),
    "rflbm_batch_lattice": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(_VP)]),
    "rflbm_batch_set_params": (ctypes.c_int, [_VP, ctypes.c_int32, _PP]),
    "rflbm_batch_step": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "rflbm_batch_step_separate": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "rflbm_batch_sync": (ctypes.c_int, [_VP]),
    "rflbm_batch_step_count": (ctypes.c_int64, [_VP]),
    "rflbm_batch_set_step_count": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "rflbm_batch_stats_config": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "rflbm_batch_nodes": (ctypes.c_int64, [_VP]),
    "rflbm_batch_set_launch": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "rflbm_batch_get_launch": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]),
    "rflbm_batch_time_steps": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    "rflbm_batch_autotune": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_char_p]),
    "rflbm_rng_normals": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _VP, _VP,
                                         _VP]),
    "rflbm_copy": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, _VP]),
    "rflbm_last_error": (ctypes.c_char_p, []),
    "rflbm_version": (ctypes.c_char_p, []),
}


def load_library():
    """Loads librflbm.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first "
                          "(python -m paper_2507_08820_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != OK:
        raise RFLBMError(status, load_library().rflbm_last_error().decode())


def make_params(dims, *, storage="f32", model="reg", kT=0.0, tau=1.0, tau_bulk=None,
                tau_ghost=1.0, rho0=1.0, seed=1, stream_id=0, philox_rounds=7,
                storage_scale=0.0) -> Params:
    lib = load_library()
    p = Params()
    lib.rflbm_params_default(ctypes.byref(p), *[int(d) for d in dims])
    p.storage = STORAGE[storage]
    p.model = MODEL[model]
    p.philox_rounds = philox_rounds
    p.rho0 = rho0
    p.kT = kT
    p.tau_shear = tau
    p.tau_bulk = tau if tau_bulk is None else tau_bulk
    tg = np.broadcast_to(np.asarray(tau_ghost, dtype=np.float64), (17,))
    for k in range(17):
        p.tau_ghost[k] = float(tg[k])
    p.seed = seed
    p.stream_id = stream_id
    p.storage_scale = storage_scale
    return p


def params_kwargs(p: Params) -> dict:
    """The make_params keywords that reproduce p (the box aside)."""
    storage = {v: k for k, v in STORAGE.items()}[p.storage]
    model = {v: k for k, v in MODEL.items()}[p.model]
    return dict(storage=storage, model=model, kT=p.kT, tau=p.tau_shear, tau_bulk=p.tau_bulk,
                tau_ghost=[p.tau_ghost[k] for k in range(17)], rho0=p.rho0, seed=p.seed,
                stream_id=p.stream_id, philox_rounds=p.philox_rounds, storage_scale=p.storage_scale)


def merged_params(current: Params, dims, **changes) -> Params:
    """current with the given make_params keywords changed; every other field
    keeps its value.  A new tau without tau_bulk also sets the bulk rate when
    that rate followed the shear rate before (tau_bulk == tau)."""
    kw = params_kwargs(current)
    if "tau" in changes and "tau_bulk" not in changes and current.tau_bulk == current.tau_shear:
        kw["tau_bulk"] = None
    kw.update(changes)
    return make_params(dims, **kw)


def _torch():
    import torch
    return torch


def _dev_ptr(t) -> int:
    return int(t.data_ptr())


def _after_torch(stream, device):
    """Orders `stream` after the work torch has queued on its current stream
    (inputs it just copied, memory its caching allocator just handed out)."""
    cur = _torch().cuda.current_stream(device)
    if cur != stream:
        stream.wait_stream(cur)


def _before_torch(stream, device):
    """Orders torch's current stream after the work queued on `stream` (results
    the library wrote into tensors that torch code reads next)."""
    cur = _torch().cuda.current_stream(device)
    if cur != stream:
        cur.wait_stream(stream)


def _field(a, device, dims, rows=1):
    """A density (rows = 1) or velocity (rows = 3) field as a contiguous FP64
    device tensor of rows x N values, N = nx ny nz, in the library's node
    order n = x + nx (y + ny z).  Accepted shapes: (N,) or (nz, ny, nx) for a
    density (a scalar is broadcast), (3, N) or (3, nz, ny, nx) for a velocity
    (component first); a box-shaped array is indexed [z, y, x], so its
    flattening is the node order.  Any other shape raises ValueError before the
    library reads rows * N values."""
    nx, ny, nz = (int(d) for d in dims)
    n = nx * ny * nz
    if rows == 1 and not hasattr(a, "data_ptr") and np.ndim(a) == 0:
        a = np.full(n, float(a))
    shape = tuple(a.shape) if hasattr(a, "shape") else np.shape(a)
    box = (nz, ny, nx)
    allowed = {(n,), box} if rows == 1 else {(3, n), (3,) + box}
    if shape not in allowed:
        raise ValueError(f"field of shape {shape}; expected one of {sorted(allowed)} "
                         f"(box-shaped fields are indexed [z, y, x])")
    t = _as_device_f64(a, device)
    return t.reshape(rows, n) if rows > 1 else t.reshape(n)


def _as_device_f64(a, device):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


class Lattice:
    """A periodic D3Q27 box stepped by the Reg-FLBM kernels of librflbm."""

    def __init__(self, dims, device="cuda", stream=None, **kw):
        torch = _torch()
        self.lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.n = int(np.prod(self.dims))
        self.device = torch.device(device)
        self.params = make_params(self.dims, **kw)
        nbytes = self.lib.rflbm_required_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            # re-run create to obtain the validation message
            handle = _VP()
            check(self.lib.rflbm_create(ctypes.byref(self.params), None, 0, None,
                                        ctypes.byref(handle)))
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = _dev_ptr(self._buf)
        self._ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = _VP()
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_create(ctypes.byref(self.params), _VP(self._ptr), nbytes,
                                    _VP(self.stream.cuda_stream), ctypes.byref(self._h)))

    @classmethod
    def _view(cls, batch, r, handle, dims, params):
        """A borrowed replica of a Batch (released with the batch)."""
        self = cls.__new__(cls)
        self.lib = batch.lib
        self.dims = tuple(dims)
        self.n = int(np.prod(self.dims))
        self.device = batch.device
        self.params = params
        self.stream = batch.stream
        self._h = handle
        self._batch = batch
        self._owner = False
        return self

    # -- life cycle --------------------------------------------------------
    def close(self):
        if getattr(self, "_owner", True) and getattr(self, "_h", None) and self._h.value:
            self.lib.rflbm_destroy(self._h)
        self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- parameters and time ----------------------------------------------
    @property
    def t(self) -> int:
        return int(self.lib.rflbm_step_count(self._h))

    @t.setter
    def t(self, value: int):
        check(self.lib.rflbm_set_step_count(self._h, int(value)))

    def set_params(self, **kw):
        """Changes the given make_params keywords; the others keep their values
        (see merged_params).  Box and storage type are fixed at creation."""
        p = merged_params(self.params, self.dims, **kw)
        check(self.lib.rflbm_set_params(self._h, ctypes.byref(p)))
        self.params = p

    # -- state ---------------------------------------------------------------
    def init_equilibrium(self, rho=None, u=None):
        r = None if rho is None else _field(rho, self.device, self.dims)
        v = None if u is None else _field(u, self.device, self.dims, rows=3)
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_init_equilibrium(self._h, None if r is None else _VP(_dev_ptr(r)),
                                              None if v is None else _VP(_dev_ptr(v)), 0))
        self._keep = (r, v)  # alive until the stream has consumed them
        self.stream.synchronize()

    def init_thermal(self, rho=None, u=None):
        """f^(0)(rho, u) plus Gaussian deviations of the stationary covariance."""
        r = None if rho is None else _field(rho, self.device, self.dims)
        v = None if u is None else _field(u, self.device, self.dims, rows=3)
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_init_thermal(self._h, None if r is None else _VP(_dev_ptr(r)),
                                          None if v is None else _VP(_dev_ptr(v)), 0))
        self._keep = (r, v)
        self.stream.synchronize()

    def populations(self):
        """f(x, t) as a (27, N) float64 tensor on the device."""
        torch = _torch()
        out = torch.empty((27, self.n), dtype=torch.float64, device=self.device)
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_get_populations(self._h, _VP(_dev_ptr(out)), 0))
        _before_torch(self.stream, self.device)
        return out

    def populations_at(self, nodes):
        """f(x, t) at the given node indices as a (27, len(nodes)) float64 tensor
        on the device (indices are checked against the box on the host)."""
        torch = _torch()
        idx = np.ascontiguousarray(nodes, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= self.n):
            raise ValueError("node index outside the box")
        nd = torch.as_tensor(idx.astype(np.uint32), device=self.device)
        out = torch.empty((27, idx.size), dtype=torch.float64, device=self.device)
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_get_populations_at(self._h, _VP(_dev_ptr(nd)), int(idx.size),
                                                _VP(_dev_ptr(out))))
        self.stream.synchronize()
        return out

    def set_populations(self, f):
        d = _as_device_f64(f, self.device).reshape(27, self.n)
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_set_populations(self._h, _VP(_dev_ptr(d)), 0))
        self.stream.synchronize()

    def moments(self, mask=M_RHO | M_J | M_PI):
        torch = _torch()
        nf = (1 if mask & M_RHO else 0) + (3 if mask & M_J else 0) + (6 if mask & M_PI else 0)
        out = torch.empty((nf, self.n), dtype=torch.float32, device=self.device)
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_get_moments(self._h, mask, _VP(_dev_ptr(out)), 0))
        _before_torch(self.stream, self.device)
        return out

    def moments_host_noalloc(self, mask=M_RHO | M_J | M_PI):
        """The moment fields as a host (numpy) array, staged through the
        library's fixed device array: no device memory is allocated."""
        import numpy as np
        nf = (1 if mask & M_RHO else 0) + (3 if mask & M_J else 0) + (6 if mask & M_PI else 0)
        out = np.empty((nf, self.n), dtype=np.float32)
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_get_moments_host_noalloc(self._h, mask, _VP(out.ctypes.data)))
        return out

    # -- stepping --------------------------------------------------------------
    def step(self, nsteps=1):
        check(self.lib.rflbm_step(self._h, int(nsteps)))

    def sync(self):
        check(self.lib.rflbm_sync(self._h))

    def set_launch(self, bx, xcd_remap=True):
        check(self.lib.rflbm_set_launch(self._h, int(bx), int(bool(xcd_remap))))

    def get_launch(self):
        bx, remap = ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.rflbm_get_launch(self._h, ctypes.byref(bx), ctypes.byref(remap)))
        return bx.value, bool(remap.value)

    def set_row_blocks(self, enable=True):
        check(self.lib.rflbm_set_row_blocks(self._h, int(bool(enable))))

    @property
    def row_blocks(self) -> bool:
        """True when odd steps run in whole-row blocks (aligned full-line loads and
        stores: FP32 storage, or k_BT = 0, with n_x a multiple of 64 up to 1024).
        Even steps of such lattices run in one-wave x-segments."""
        active = ctypes.c_int32()
        check(self.lib.rflbm_get_row_blocks(self._h, ctypes.byref(active)))
        return bool(active.value)

    def time_steps(self, nsteps) -> float:
        ms = ctypes.c_double()
        check(self.lib.rflbm_time_steps(self._h, int(nsteps), ctypes.byref(ms)))
        return ms.value

    # -- observables -----------------------------------------------------------
    def stats_config(self, every):
        check(self.lib.rflbm_stats_config(self._h, int(every)))

    def stats(self) -> dict:
        s = Stats()
        check(self.lib.rflbm_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        check(self.lib.rflbm_reset_stats(self._h))

    def sk_sample(self):
        check(self.lib.rflbm_sk_sample(self._h))

    def sk(self, field):
        ns = self.lib.rflbm_sk_nshells(self._h)
        sums = np.zeros(ns)
        counts = np.zeros(ns, dtype=np.int64)
        samples = ctypes.c_int64()
        idx = FIELDS.index(field) if isinstance(field, str) else int(field)
        check(self.lib.rflbm_get_sk(self._h, idx, sums.ctypes.data_as(_VP), counts.ctypes.data_as(_VP),
                                    ns, ctypes.byref(samples)))
        return sums, counts, samples.value

    def reset_sk(self):
        check(self.lib.rflbm_reset_sk(self._h))


class Batch:
    """Independent replicas (own box, taus, kT, rho0, seed, stream id) stepped
    together by one persistent launch per step.  ``replicas`` is a list of
    dicts with ``dims`` plus any keyword of make_params."""

    def __init__(self, replicas, device="cuda", stream=None, **common):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.device(device)
        self.replicas = [dict(r) for r in replicas]
        n = len(self.replicas)
        arr = (Params * n)()
        for i, r in enumerate(self.replicas):
            kw = dict(common)
            kw.update({k: v for k, v in r.items() if k != "dims"})
            arr[i] = make_params(r["dims"], **kw)
        self.params = arr
        nbytes = self.lib.rflbm_batch_required_bytes(n, arr)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = _VP()
        if nbytes == 0:
            check(self.lib.rflbm_batch_create(n, arr, None, 0, None, ctypes.byref(self._h)))
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (_dev_ptr(self._buf) + 255) // 256 * 256
        _after_torch(self.stream, self.device)
        check(self.lib.rflbm_batch_create(n, arr, _VP(ptr), nbytes, _VP(self.stream.cuda_stream),
                                          ctypes.byref(self._h)))
        self.views = []
        for i, r in enumerate(self.replicas):
            h = _VP()
            check(self.lib.rflbm_batch_lattice(self._h, i, ctypes.byref(h)))
            self.views.append(Lattice._view(self, i, h, r["dims"], arr[i]))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            for v in self.views:
                v._h = _VP()
            self.lib.rflbm_batch_destroy(self._h)
            self._h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.views)

    def __getitem__(self, r):
        return self.views[r]

    @property
    def t(self) -> int:
        return int(self.lib.rflbm_batch_step_count(self._h))

    @t.setter
    def t(self, value):
        check(self.lib.rflbm_batch_set_step_count(self._h, int(value)))

    @property
    def nodes(self) -> int:
        return int(self.lib.rflbm_batch_nodes(self._h))

    def set_params(self, r, **kw):
        """Changes the given make_params keywords of replica r; the others keep
        their values (see merged_params)."""
        p = merged_params(self.views[r].params, self.replicas[r]["dims"], **kw)
        check(self.lib.rflbm_batch_set_params(self._h, int(r), ctypes.byref(p)))
        self.views[r].params = p

    def step(self, nsteps=1):
        check(self.lib.rflbm_batch_step(self._h, int(nsteps)))

    def step_separate(self, nsteps=1):
        check(self.lib.rflbm_batch_step_separate(self._h, int(nsteps)))

    def sync(self):
        check(self.lib.rflbm_batch_sync(self._h))

    def stats_config(self, every):
        """Statistics of every replica on every `every`-th step (0: off); read
        them with stats() on a replica view."""
        check(self.lib.rflbm_batch_stats_config(self._h, int(every)))

    def set_launch(self, tile=256, blocks_per_cu=8, graph_steps=0):
        check(self.lib.rflbm_batch_set_launch(self._h, int(tile), int(blocks_per_cu),
                                              int(graph_steps)))

    def get_launch(self):
        t, b, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.rflbm_batch_get_launch(self._h, ctypes.byref(t), ctypes.byref(b),
                                              ctypes.byref(g)))
        return t.value, b.value, g.value

    def time_steps(self, nsteps) -> float:
        ms = ctypes.c_double()
        check(self.lib.rflbm_batch_time_steps(self._h, int(nsteps), ctypes.byref(ms)))
        return ms.value

    def autotune(self, trial_steps=10, cache_path=None):
        check(self.lib.rflbm_batch_autotune(self._h, int(trial_steps),
                                            None if cache_path is None else
                                            str(cache_path).encode()))
        return self.get_launch()


def rng_normals(seed, stream_id, rounds, node0, count, t, device="cuda"):
    """The uniforms and normals the step kernel draws (each (count, 24) float32)."""
    torch = _torch()
    lib = load_library()
    u = torch.empty((count, 24), dtype=torch.float32, device=device)
    z = torch.empty((count, 24), dtype=torch.float32, device=device)
    s = torch.cuda.current_stream(device)
    check(lib.rflbm_rng_normals(seed, stream_id, rounds, node0, count, t, _VP(_dev_ptr(u)),
                                _VP(_dev_ptr(z)), _VP(s.cuda_stream)))
    s.synchronize()
    return u, z


def copy(dst, src, nbytes, stream=None):
    """Copies nbytes from tensor src to tensor dst with the library's copy
    kernel (bandwidth reference); both must hold at least nbytes."""
    torch = _torch()
    for t in (dst, src):
        if not t.is_contiguous() or int(nbytes) > t.numel() * t.element_size():
            raise ValueError("copy needs contiguous tensors of at least nbytes")
    s = stream if stream is not None else torch.cuda.current_stream(dst.device)
    check(load_library().rflbm_copy(_VP(_dev_ptr(dst)), _VP(_dev_ptr(src)), int(nbytes),
                                    _VP(s.cuda_stream)))
