"""Python binding of the C ABI in include/lbf.h (argument marshalling only).

Every step of the update runs in the HIP kernels of ``liblbf.so``; torch is
used for device memory and streams.  If the library has not been built, or
no GPU is present, the calls raise: there is no fallback path.
"""
import ctypes
import os
import warnings

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbf.so")

LB_OK, LB_EINVAL, LB_EDEVICE, LB_ESTATE, LB_EUNSUPPORTED = 0, -1, -2, -3, -4
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
STORAGE_DTYPE = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
INIT = {"rest": 0, "thermal": 1, "fields": 2, "keep": 3}
THERMAL_MODES = {"all": 0, "stress_only": 1}
LATTICE = {"d3q19": 0, "d2q9": 1}
LATTICE_QD = {"d3q19": (19, 3), "d2q9": (9, 2)}  # populations q, dimension d


class LbParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("kT", ctypes.c_double),
        ("gamma_bulk", ctypes.c_double), ("gamma_shear", ctypes.c_double),
        ("gamma_odd", ctypes.c_double), ("gamma_even", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("thermal_modes", ctypes.c_int32), ("lattice", ctypes.c_int32),
    ]


class LbSchedule(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("order", ctypes.c_int32), ("graph_chunk", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32 * 2), ("tiling", ctypes.c_int32 * 2),
                ("resident", ctypes.c_int32), ("group_mb", ctypes.c_int32), ("fused", ctypes.c_int32)]


def _sched_dict(s):
    return {"block": s.block, "order": s.order, "graph_chunk": s.graph_chunk,
            "xcd_remap": list(s.xcd_remap), "tiling": list(s.tiling),
            "resident": s.resident, "group_mb": s.group_mb, "fused": s.fused}


def _pair(v):
    """An int (both parities) or an (even, odd) pair."""
    if isinstance(v, (list, tuple)):
        return (ctypes.c_int32 * 2)(int(v[0]), int(v[1]))
    return (ctypes.c_int32 * 2)(int(v), int(v))


def _make_schedule(block, order, xcd_remap, graph_chunk, tiling, resident=0, group_mb=0, fused=0):
    return LbSchedule(int(block), int(order), int(graph_chunk), _pair(xcd_remap), _pair(tiling),
                      int(resident), int(group_mb), int(fused))


# (name, restype, argtypes) of every entry point in include/lbf.h
_P = ctypes.POINTER
_vp = ctypes.c_void_p
SIGNATURES = [
    ("lb_state_bytes", ctypes.c_size_t, [_P(LbParams)]),
    ("lb_init", ctypes.c_int, [_P(LbParams), _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64, _P(_vp)]),
    ("lb_step", ctypes.c_int, [_vp, ctypes.c_int64]),
    ("lb_propagate", ctypes.c_int, [_vp, ctypes.c_int64]),
    ("lb_populations", ctypes.c_int, [_vp, _vp]),
    ("lb_moments", ctypes.c_int, [_vp, _vp]),
    ("lb_modes", ctypes.c_int, [_vp, _vp]),
    ("lb_check", ctypes.c_int, [_vp, _P(ctypes.c_int64), _P(ctypes.c_double)]),
    ("lb_step_count", ctypes.c_int64, [_vp]),
    ("lb_destroy", None, [_vp]),
    ("lb_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("lb_last_error", ctypes.c_char_p, []),
    ("lb_params_from_physical", ctypes.c_int, [ctypes.c_double] * 6 + [_P(LbParams)]),
    ("lb_batch_pool_bytes", ctypes.c_size_t, [_P(LbParams), ctypes.c_int32]),
    ("lb_batch_offset", ctypes.c_size_t, [_P(LbParams), ctypes.c_int32, ctypes.c_int32]),
    ("lb_batch_init", ctypes.c_int, [_P(LbParams), ctypes.c_int32, _vp, _vp, ctypes.c_int32,
                                     ctypes.c_int64, _P(_vp)]),
    ("lb_batch_step", ctypes.c_int, [_vp, ctypes.c_int64]),
    ("lb_batch_view", ctypes.c_int, [_vp, ctypes.c_int32, _P(_vp)]),
    ("lb_get_schedule", ctypes.c_int, [_vp, _P(LbSchedule)]),
    ("lb_set_schedule", ctypes.c_int, [_vp, _P(LbSchedule)]),
    ("lb_autotune", ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_char_p, ctypes.c_size_t]),
    ("lb_copy_rate", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int32, _vp, _P(ctypes.c_double)]),
    ("lb_step_noalloc", ctypes.c_int, [_P(LbParams), ctypes.c_int32, _vp, _vp, ctypes.c_int64, ctypes.c_int64]),
]
NOALLOC_MAX_REPLICAS = 64

_lib = None


def lib():
    """The loaded liblbf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class LBError(RuntimeError):
    def __init__(self, code, where):
        L = lib()
        msg = L.lb_last_error().decode()
        super().__init__(f"{where}: {L.lb_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(rc, where):
    if rc != LB_OK:
        raise LBError(rc, where)


def make_params(nx, ny, nz, storage="f32", rho0=1.0, kT=0.0, gamma_bulk=0.5, gamma_shear=0.5,
                gamma_odd=0.0, gamma_even=0.0, seed=0, thermal_modes="all", lattice="d3q19"):
    return LbParams(int(nx), int(ny), int(nz), STORAGE[storage], float(rho0), float(kT),
                    float(gamma_bulk), float(gamma_shear), float(gamma_odd), float(gamma_even),
                    int(seed), THERMAL_MODES[thermal_modes], LATTICE[lattice])


def physical_params(b, h, rho, eta, zeta, kBT, lattice="d3q19"):
    """Lattice rho0, kT, gamma_shear, gamma_bulk from physical spacing, time
    step, density, viscosities and k_B T (Sec. VI), via the C ABI; the
    lattice fixes the dimension d."""
    p = make_params(1, 1, 1, lattice=lattice)
    _check(lib().lb_params_from_physical(b, h, rho, eta, zeta, kBT, ctypes.byref(p)),
           "lb_params_from_physical")
    return dict(rho0=p.rho0, kT=p.kT, gamma_shear=p.gamma_shear, gamma_bulk=p.gamma_bulk)


def copy_rate(gib=4, reps=10, device="cuda", stream=None):
    """GB/s (read + write) of the library's float4 non-temporal device copy
    of two gib-GiB buffers: the practical streaming ceiling."""
    dev = torch.device(device)
    n = int(gib * (1 << 30)) // 16 * 16
    src = torch.ones(n // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    sp, s = _stream_ptr(dev, stream)
    _adopt(src, dev, s)
    _adopt(dst, dev, s)
    out = ctypes.c_double(0.0)
    _check(lib().lb_copy_rate(_aligned(src), _aligned(dst), n, int(reps), sp, ctypes.byref(out)), "lb_copy_rate")
    del src, dst
    return out.value


def step_noalloc(replicas, pool, t0, nsteps, storage="f32", lattice="d3q19", stream=None):
    """lb_step_noalloc: advance the lattices `replicas` (dicts of make_params
    keywords) whose states lie in the device tensor `pool` (laid out as for
    an Ensemble; one state for a single lattice) from step t0 by nsteps
    steps, with no context and no device allocation."""
    params = [make_params(storage=storage, lattice=lattice, **r) for r in replicas]
    arr = (LbParams * len(params))(*params)
    dev = pool.device
    sp, s = _stream_ptr(dev, stream)
    _adopt(pool, dev, s)
    _check(lib().lb_step_noalloc(arr, len(params), _aligned(pool), sp, int(t0), int(nsteps)), "lb_step_noalloc")
    cur = torch.cuda.current_stream(dev)
    if s != cur:
        cur.wait_stream(s)


def _stream_ptr(device, stream):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream), s


def _adopt(t, device, lat_stream):
    """Order the library's work on lat_stream after the caller's current
    stream (which may have just produced or recycled t's memory), and keep
    the caching allocator from reusing t's memory before lat_stream is done
    with it."""
    cur = torch.cuda.current_stream(device)
    if lat_stream != cur:
        lat_stream.wait_stream(cur)
        t.record_stream(lat_stream)


def _aligned(t):
    if t.data_ptr() % 256:
        raise ValueError("device buffers must be 256-byte aligned")
    return ctypes.c_void_p(t.data_ptr())


class _Gathers:
    """Parity-resolved gathers shared by lattices and replica views."""

    def _dims(self):
        return self.nz, self.ny, self.nx

    @property
    def q(self):
        return LATTICE_QD[self.lattice][0]

    @property
    def dim(self):
        return LATTICE_QD[self.lattice][1]

    def _gather(self, fn, name, rows):
        """Run a gather on the lattice's stream into a new tensor that the
        caller's current stream may use at once."""
        lat_stream = self.stream if isinstance(self, Lattice) else self._ens.stream
        out = torch.empty((rows, *self._dims()), dtype=torch.float32, device=self.device)
        _adopt(out, self.device, lat_stream)
        _check(fn(self._ctx, _aligned(out)), name)
        cur = torch.cuda.current_stream(self.device)
        if lat_stream != cur:
            cur.wait_stream(lat_stream)
        return out

    def populations(self):
        return self._gather(lib().lb_populations, "lb_populations", self.q)

    def moments(self):
        """(1 + d, nz, ny, nx): rho, jx, jy[, jz]."""
        return self._gather(lib().lb_moments, "lb_moments", 1 + self.dim)

    def modes(self):
        return self._gather(lib().lb_modes, "lb_modes", self.q)

    def check(self):
        """(n_bad, [sum rho, sum jx, sum jy, sum jz]); raises on LB_ESTATE."""
        n_bad = ctypes.c_int64(0)
        sums = (ctypes.c_double * 4)()
        rc = lib().lb_check(self._ctx, ctypes.byref(n_bad), sums)
        if rc not in (LB_OK, LB_ESTATE):
            _check(rc, "lb_check")
        return int(n_bad.value), list(sums)

    @property
    def t(self):
        return int(lib().lb_step_count(self._ctx))


class Lattice(_Gathers):
    """One periodic lattice (D3Q19, or D2Q9 with nz = 1); the state is a
    caller-owned torch tensor (q, nz, ny, nx) of scaled deviations in the
    storage dtype."""

    def __init__(self, nx, ny, nz, storage="f32", rho0=1.0, kT=0.0, gamma_bulk=0.5,
                 gamma_shear=0.5, gamma_odd=0.0, gamma_even=0.0, seed=0, thermal_modes="all",
                 init="rest", fields=None, t0=0, device="cuda", stream=None, state=None,
                 lattice="d3q19"):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.storage = storage
        self.lattice = lattice
        self.params = make_params(nx, ny, nz, storage, rho0, kT, gamma_bulk, gamma_shear,
                                  gamma_odd, gamma_even, seed, thermal_modes, lattice)
        self.device = torch.device(device)
        nbytes = lib().lb_state_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            raise LBError(LB_EINVAL, "lb_state_bytes")
        shape = (self.q, self.nz, self.ny, self.nx)
        if state is None:
            state = torch.empty(shape, dtype=STORAGE_DTYPE[storage], device=self.device)
        if tuple(state.shape) != shape or state.dtype != STORAGE_DTYPE[storage] or not state.is_contiguous():
            raise ValueError("state must be a contiguous (q, nz, ny, nx) tensor of the storage dtype")
        self.state = state
        f = None
        if init == "fields":
            fshape = (1 + self.dim, self.nz, self.ny, self.nx)
            if fields is None:
                raise ValueError(f"init='fields' needs fields {fshape}")
            self._fields = fields.to(device=self.device, dtype=torch.float32).contiguous()
            if tuple(self._fields.shape) != fshape:
                raise ValueError(f"fields must be {fshape}")
            f = _aligned(self._fields)
        sp, self.stream = _stream_ptr(self.device, stream)
        _adopt(self.state, self.device, self.stream)
        if f is not None:
            _adopt(self._fields, self.device, self.stream)
        ctx = ctypes.c_void_p()
        _check(lib().lb_init(ctypes.byref(self.params), _aligned(self.state), sp, INIT[init], f,
                             int(t0), ctypes.byref(ctx)), "lb_init")
        self._ctx = ctx
        if storage == "bf16" and kT == 0:
            warnings.warn(lib().lb_last_error().decode(), stacklevel=2)

    def step(self, n=1):
        _check(lib().lb_step(self._ctx, int(n)), "lb_step")

    def propagate(self, n=1):
        """n propagation-only steps (no collision; an exact permutation)."""
        _check(lib().lb_propagate(self._ctx, int(n)), "lb_propagate")

    def schedule(self):
        s = LbSchedule()
        _check(lib().lb_get_schedule(self._ctx, ctypes.byref(s)), "lb_get_schedule")
        return _sched_dict(s)

    def set_schedule(self, block=256, order=0, xcd_remap=1, graph_chunk=16, tiling=0, resident=0, group_mb=0,
                     fused=0):
        """xcd_remap and tiling: an int for both step parities or an
        (even, odd) pair; resident: cache every access (1) or stream (0);
        group_mb: replica groups of at most this many MiB of state (0: one);
        fused: two steps per launch through a second buffer (1) or one
        in-place step per launch (0)."""
        s = _make_schedule(block, order, xcd_remap, graph_chunk, tiling, resident, group_mb, fused)
        _check(lib().lb_set_schedule(self._ctx, ctypes.byref(s)), "lb_set_schedule")

    def autotune(self, steps=10):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().lb_autotune(self._ctx, int(steps), buf, len(buf)), "lb_autotune")
        return buf.value.decode()

    def close(self):
        if getattr(self, "_ctx", None):
            lib().lb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ReplicaView(_Gathers):
    def __init__(self, ens, r, ctx):
        p = ens.params[r]
        self.nx, self.ny, self.nz = p.nx, p.ny, p.nz
        self.lattice = ens.lattice
        self.device = ens.device
        self._ctx = ctx
        self._ens = ens

    def close(self):
        if getattr(self, "_ctx", None):
            lib().lb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Independent replicas (own box, rates, kT, seed; one storage type and
    one lattice) advanced together, one kernel launch per step (per replica group) for all of
    them."""

    def __init__(self, replicas, storage="f32", init="thermal", t0=0, device="cuda", stream=None,
                 lattice="d3q19"):
        self.storage = storage
        self.lattice = lattice
        self.device = torch.device(device)
        self.params = [make_params(storage=storage, lattice=lattice, **r) for r in replicas]
        n = len(self.params)
        self._arr = (LbParams * n)(*self.params)
        nbytes = lib().lb_batch_pool_bytes(self._arr, n)
        if nbytes == 0:
            raise LBError(LB_EINVAL, "lb_batch_pool_bytes")
        self.pool = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        sp, self.stream = _stream_ptr(self.device, stream)
        _adopt(self.pool, self.device, self.stream)
        ctx = ctypes.c_void_p()
        _check(lib().lb_batch_init(self._arr, n, _aligned(self.pool), sp, INIT[init], int(t0),
                                   ctypes.byref(ctx)), "lb_batch_init")
        self._ctx = ctx
        self._views = {}

    def __len__(self):
        return len(self.params)

    def sites(self):
        return sum(p.nx * p.ny * p.nz for p in self.params)

    def step(self, n=1):
        _check(lib().lb_batch_step(self._ctx, int(n)), "lb_batch_step")

    def propagate(self, n=1):
        """n propagation-only steps of every replica (no collision)."""
        _check(lib().lb_propagate(self._ctx, int(n)), "lb_propagate")

    @property
    def t(self):
        return int(lib().lb_step_count(self._ctx))

    def view(self, r):
        if r not in self._views:
            v = ctypes.c_void_p()
            _check(lib().lb_batch_view(self._ctx, int(r), ctypes.byref(v)), "lb_batch_view")
            self._views[r] = ReplicaView(self, r, v)
        return self._views[r]

    def replica_state(self, r):
        """The raw state tensor of replica r (a view into the pool)."""
        p = self.params[r]
        off = lib().lb_batch_offset(self._arr, len(self.params), int(r))
        nbytes = lib().lb_state_bytes(ctypes.byref(p))
        q = LATTICE_QD[self.lattice][0]
        return self.pool[off:off + nbytes].view(STORAGE_DTYPE[self.storage]).view(q, p.nz, p.ny, p.nx)

    def schedule(self):
        s = LbSchedule()
        _check(lib().lb_get_schedule(self._ctx, ctypes.byref(s)), "lb_get_schedule")
        return _sched_dict(s)

    def set_schedule(self, block=256, order=0, xcd_remap=1, graph_chunk=16, tiling=0, resident=0, group_mb=0,
                     fused=0):
        """xcd_remap and tiling: an int for both step parities or an
        (even, odd) pair; resident: cache every access (1) or stream (0);
        group_mb: replica groups of at most this many MiB of state (0: one);
        fused: two steps per launch through a second buffer (1) or one
        in-place step per launch (0)."""
        s = _make_schedule(block, order, xcd_remap, graph_chunk, tiling, resident, group_mb, fused)
        _check(lib().lb_set_schedule(self._ctx, ctypes.byref(s)), "lb_set_schedule")

    def autotune(self, steps=10):
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().lb_autotune(self._ctx, int(steps), buf, len(buf)), "lb_autotune")
        return buf.value.decode()

    def close(self):
        for v in self._views.values():
            v.close()
        self._views = {}
        if getattr(self, "_ctx", None):
            lib().lb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
